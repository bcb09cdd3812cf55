"""Pins of the oracle's propagation in an inhomogeneous field (Sect. 3: the
precise extrapolation to a chamber accounts for the field; the paper gives
no map, so the field model is synthetic: Bz(r, z) = Bz0 (1 + b_r (r/370)^2 +
b_z (z/360)^2)).

The truth comes from the generator, which integrates the equation of motion
in the GLOBAL frame (position, direction azimuth, transverse path length as
the variable, 0.25 cm Runge-Kutta steps in extended precision, Newton onto
each plane).  The oracle integrates in each SECTOR frame with local x as the
variable over steps of at most field_step.  The two share no code.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import synth

FLOORS = np.array([10.0, 10.0, 0.1, 0.1, 0.1])


def _noise_free(P, n, seed, dtype=np.longdouble):
    g = synth.generate_group(np.random.default_rng(seed), P, n, noise_free=True, ms=False, fp32=False,
                             fake_ratio=0.0, dtype=dtype)
    w = synth._concat_groups([g], P)
    for k in ("tkl_y", "tkl_z", "tkl_dy"):
        w[k] = np.zeros(0)
    w["tkl_det_row"] = np.zeros(0, np.uint32)
    w["tkl_group"] = np.zeros(0, np.int32)
    w["p"] = g["truth_seed"]
    return w


def _worst(P, w, min_ok=150):
    o = O.match(P, w, layers=True, threads=2)
    T = w["truth"]
    worst = 0.0
    for l in range(6):
        ok = (T["sec"][l] >= 0) & (o["lsec"][l] == T["sec"][l]) & (o["flags"] == 0)
        assert ok.sum() > min_ok
        for k, name in enumerate(("y", "z", "snp", "tgl", "qpt")):
            e = np.abs(o["lp"][l, k, ok] - T[name][l, ok].astype(np.float64)) / \
                np.maximum(np.abs(T[name][l, ok].astype(np.float64)), FLOORS[k])
            worst = max(worst, float(e.max()))
    return worst


@pytest.mark.parametrize("field", [(-0.02, -0.04), (0.03, 0.05)])
def test_runge_kutta_lands_on_the_integrated_crossings(field):
    """Noise-free tracks in the field model: the oracle's local-frame steps
    (0.25 cm) with sector hops land on the generator's global-frame crossings
    at all six layers within 1e-9 (relative, floors 10 cm, 0.1)."""
    P = synth.default_params(x_over_x0=0.0, **synth.field_map_overrides(*field))
    w = _noise_free(P, 300, 31)
    assert _worst(P, w) < 1e-9


def test_the_field_matters():
    """Sensitivity: the same truth propagated as if the field were uniform
    misses the crossings by far more than the tolerance (so the pin above
    tests the map, its radius and its z dependence)."""
    P = synth.default_params(x_over_x0=0.0, **synth.field_map_overrides())
    w = _noise_free(P, 300, 32)
    U = dict(P, field_br=0.0, field_bz=0.0)
    assert _worst(U, w, min_ok=100) > 1e-5
    Pr = dict(P, field_bz=0.0)     # the z dependence alone dropped
    assert _worst(Pr, w, min_ok=100) > 1e-7


def test_step_size_converges():
    """The integration error falls with the step as a 4th-order method's
    does (halving the step divides it by about 16) down to 1e-9 at 0.25 cm."""
    P = synth.default_params(x_over_x0=0.0, **synth.field_map_overrides(0.05, 0.08))
    w = _noise_free(P, 200, 33)
    e1 = _worst(dict(P, field_step=1.0), w)
    e05 = _worst(dict(P, field_step=0.5), w)
    e025 = _worst(dict(P, field_step=0.25), w)
    assert e025 < 1e-9 and 8 < e1 / e05 < 32 and 8 < e05 / e025 < 32, (e1, e05, e025)


def test_uniform_map_equals_the_closed_form():
    """A map with zero coefficients is the uniform field: the closed-form step
    (the Runge-Kutta path is only taken for a non-uniform map); and a tiny
    non-uniformity changes the state by a correspondingly tiny amount."""
    P = synth.default_params(x_over_x0=0.0)
    w = _noise_free(P, 200, 34)
    a = O.match(P, w, layers=True, threads=2)
    b = O.match(dict(P, field_br=1e-12, field_bz=1e-12), w, layers=True, threads=2)
    ok = np.isfinite(a["lp"]) & np.isfinite(b["lp"])
    assert np.abs(a["lp"][ok] - b["lp"][ok]).max() < 1e-8


def test_covariance_transport_matches_monte_carlo_in_the_field():
    """The covariance of the Runge-Kutta step (helix Jacobians in the local
    field of each sub-step) against the sample covariance of 40k states
    propagated through the same step."""
    P = synth.default_params(x_over_x0=0.0, **synth.field_map_overrides(0.05, 0.08))
    p0 = np.array([12.0, 150.0, 0.3, 0.7, 1.8])
    sig = np.array([0.05, 0.1, 2e-3, 2e-3, 0.02])
    C0 = np.diag(sig ** 2)
    pk = C0[np.triu_indices(5)]
    ok, p, cov, x, _ = O.propagate(P, p0.copy(), pk.copy(), 300.0, 340.0)
    assert ok
    rng = np.random.default_rng(5)
    S = p0[:, None] + rng.standard_normal((5, 40000)) * sig[:, None]
    out = np.array([O.propagate(P, S[:, i].copy(), None, 300.0, 340.0)[1] for i in range(S.shape[1])]).T
    emp = np.cov(out)
    C = np.zeros((5, 5))
    C[np.triu_indices(5)] = cov
    C = C + C.T - np.diag(np.diag(C))
    d = np.sqrt(np.diag(C))
    rel = np.abs(emp - C) / np.outer(d, d)
    assert rel.max() < 0.03, rel.max()
