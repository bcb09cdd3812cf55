"""Pins of the oracle's single steps against closed forms and textbook identities.

Nothing here compares the oracle with itself: propagation is checked against
the generator's global circle/plane crossings (computed in extended precision),
Jacobians against complex-step derivatives of an analytic rewrite of the helix
map, the transported covariance against a Monte-Carlo sample, scattering
against an angle-kick model, the Kalman update against the information form.
"""
import json
import math
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "closed_forms.json")))
KAPPA = 2.99792458e-3


def rel_state(a, b):
    """Per-component relative error with floors (y, z: 10 cm; snp, tgl: 0.1; q/pT: 0.1)."""
    floors = np.array([10.0, 10.0, 0.1, 0.1, 0.1])
    a, b = np.asarray(a), np.asarray(b)
    return np.abs(a - b) / np.maximum(np.abs(b), floors[: len(b)])


def _params(**kw):
    return synth.default_params(**kw)


def test_closed_form_layer_crossings():
    """Noise-free helices: the oracle's stepping (with sector hops) lands on the
    global circle/plane crossings at all six layers to 1e-12."""
    P = _params(x_over_x0=0.0)
    rng = np.random.default_rng(11)
    g = synth.generate_group(rng, P, 400, noise_free=True, ms=False, fp32=False,
                             fake_ratio=0.0, dtype=np.longdouble)
    w = synth._concat_groups([g], P)
    # no tracklets: the oracle only propagates and rotates
    for k in ("tkl_y", "tkl_z", "tkl_dy"):
        w[k] = np.zeros(0)
    w["tkl_det_row"] = np.zeros(0, np.uint32)
    w["tkl_group"] = np.zeros(0, np.int32)
    w["p"] = g["truth_seed"]
    o = O.match(P, w, layers=True, threads=1)
    T = w["truth"]
    n_cmp, worst = 0, 0.0
    floors = (10.0, 10.0, 0.1, 0.1, 0.1)
    for l in range(6):
        ok = (T["sec"][l] >= 0) & (o["lsec"][l] == T["sec"][l]) & (o["flags"] == 0)
        assert ok.sum() > 250
        for k, name in enumerate(("y", "z", "snp", "tgl", "qpt")):
            worst = max(worst, float(np.max(np.abs(o["lp"][l, k, ok] - T[name][l, ok]) /
                                            np.maximum(np.abs(T[name][l, ok]), floors[k]))))
        n_cmp += ok.sum()
    assert worst < 1e-12, worst
    # a hop into the neighbouring sector really happened for some tracks
    assert (o["lsec"][5] != w["sector"]).sum() > 0


def test_straight_line_limit():
    P = _params(bz=0.0)
    p = np.array([3.0, -20.0, 0.3, 0.4, 1.7])
    ok, p2, _, x2, J = O.propagate(P, p, None, 290.0, 320.0)
    f = math.sqrt(1 - 0.3 ** 2)
    assert ok
    assert abs(p2[0] - (3.0 + 30.0 * 0.3 / f)) < 1e-13
    assert abs(p2[1] - (-20.0 + 30.0 * 0.4 / f)) < 1e-13
    assert p2[2] == 0.3 and x2 == 320.0


def test_composition_and_reversal():
    P = _params()
    rng = np.random.default_rng(3)
    for _ in range(50):
        p = np.array([rng.uniform(-40, 40), rng.uniform(-200, 200), rng.uniform(-0.6, 0.6),
                      rng.uniform(-0.9, 0.9), rng.choice([-1, 1]) / rng.uniform(0.35, 5)])
        c = O.pack(np.diag([0.01, 0.02, 1e-6, 2e-6, 1e-4]) + 1e-7)
        ok1, pa, ca, _, _ = O.propagate(P, p, c, 290.0, 310.0)
        ok2, pb, cb, _, _ = O.propagate(P, pa, ca, 310.0, 355.0)
        ok3, pc, cc, _, _ = O.propagate(P, p, c, 290.0, 355.0)
        assert ok1 and ok2 and ok3
        assert rel_state(pb, pc).max() < 1e-12
        sc = np.sqrt(np.outer(np.diag(O.unpack(cc)), np.diag(O.unpack(cc))))
        assert (np.abs(O.unpack(cb) - O.unpack(cc)) / sc).max() < 1e-12
        ok4, pr, cr, xr, _ = O.propagate(P, pc, cc, 355.0, 290.0)
        assert ok4 and xr == 290.0
        assert rel_state(pr, p).max() < 1e-12
        sc0 = np.sqrt(np.outer(np.diag(O.unpack(c)), np.diag(O.unpack(c))))
        assert (np.abs(O.unpack(cr) - O.unpack(c)) / sc0).max() < 1e-10


@pytest.mark.parametrize("side", [+1, -1])
def test_reach_threshold_closed_form(side):
    """A track from the origin reaches the plane x = 290 cm (at the point where
    the plane touches the circle) iff 2R >= 290 cm."""
    gold = GOLD["reach_pt_threshold_gev_x290_bz0.5"]["value"]
    P = _params(snp_max=1.0)
    R = 145.0 * (1.0 + side * 1e-6)
    pt = KAPPA * 0.5 * R
    assert abs(KAPPA * 0.5 * 145.0 - gold) / gold < 1e-4
    xs = 250.0
    # circle through the origin centred at (R, 0) in this frame, positive track
    # (clockwise in Bz > 0): y = sqrt(R^2 - (x-R)^2), sin(phi) = (R - x)/R
    p = np.array([math.sqrt(R * R - (xs - R) ** 2), 0.0, (R - xs) / R, 0.0, 1.0 / pt])
    ok, p2, _, _, _ = O.propagate(P, p, None, xs, 290.0)
    assert ok == (side > 0)
    if ok:
        assert abs(p2[2] - (R - 290.0) / R) < 1e-12
        assert abs(p2[0] - math.sqrt(R * R - (290.0 - R) ** 2)) < 1e-9


def _helix_rewrite(p, dx, k):
    """Analytic form of the helix map (complex arithmetic allowed):
    y2 = y1 + (f1 - f2)/C, arc = (asin s2 - asin s1)/C, z2 = z1 + t arc."""
    y, z, s, t, c = p
    cu = k * c
    s2 = s + cu * dx
    f1, f2 = np.sqrt(1 - s * s), np.sqrt(1 - s2 * s2)
    arc = (np.arcsin(s2) - np.arcsin(s)) / cu
    return np.array([y + (f1 - f2) / cu, z + t * arc, s2, t, c])


def test_jacobian_complex_step():
    P = _params()
    k = -KAPPA * P["bz"]
    rng = np.random.default_rng(5)
    for _ in range(100):
        p = np.array([rng.uniform(-40, 40), rng.uniform(-200, 200), rng.uniform(-0.7, 0.7),
                      rng.uniform(-1, 1), rng.choice([-1, 1]) / rng.uniform(0.3, 3)])
        dx = rng.uniform(5, 60)
        ok, _, _, _, J = O.propagate(P, p, None, 300.0, 300.0 + dx, want_j=True)
        assert ok
        h = 1e-30
        Jc = np.zeros((5, 5))
        for j in range(5):
            pc = p.astype(complex)
            pc[j] += 1j * h
            Jc[:, j] = _helix_rewrite(pc, dx, k).imag / h
        scale = np.maximum(np.abs(Jc), 1.0)
        assert (np.abs(J - Jc) / scale).max() < 1e-11, (J, Jc)


def test_jacobian_small_curvature_limits():
    """At vanishing curvature the entries reach their straight-line limits."""
    P = _params()
    k = -KAPPA * P["bz"]
    s, t, dx = 0.4, 0.7, 30.0
    f = math.sqrt(1 - s * s)
    ok, _, _, _, J = O.propagate(P, np.array([0, 0, s, t, 1e-12]), None, 300.0, 300.0 + dx)
    assert ok
    assert abs(J[0, 2] - dx / f ** 3) < 1e-9 * dx / f ** 3
    assert abs(J[0, 4] / k - dx * dx / (2 * f ** 3)) < 1e-6
    assert abs(J[1, 4] / k - t * s * dx * dx / (2 * f ** 3)) < 1e-6


def test_rotation_roundtrip_and_invariants():
    P = _params()
    rng = np.random.default_rng(8)
    da = 2 * math.pi / 18
    for _ in range(50):
        p = np.array([rng.uniform(-50, 50), rng.uniform(-100, 100), rng.uniform(-0.5, 0.5),
                      rng.uniform(-1, 1), rng.choice([-1, 1]) / rng.uniform(0.3, 3)])
        x = 300.0
        c = O.pack(np.diag([0.01, 0.02, 1e-6, 2e-6, 1e-4]))
        ok, p1, c1, x1, J1 = O.rotate(P, p, c, x, da)
        assert ok
        # the global point and direction do not change
        a0 = 0.3
        X0, Y0 = x * math.cos(a0) - p[0] * math.sin(a0), x * math.sin(a0) + p[0] * math.cos(a0)
        X1, Y1 = x1 * math.cos(a0 + da) - p1[0] * math.sin(a0 + da), x1 * math.sin(a0 + da) + p1[0] * math.cos(a0 + da)
        assert abs(X0 - X1) < 1e-11 and abs(Y0 - Y1) < 1e-11
        assert abs((a0 + math.asin(p[2])) - (a0 + da + math.asin(p1[2]))) < 1e-12
        # rotating back restores the state; the covariance returns after
        # transporting back to the original x (first-order Jacobians compose)
        ok, p2, c2, x2, J2 = O.rotate(P, p1, c1, x1, -da)
        assert ok
        assert abs(x2 - x) < 1e-11 and rel_state(p2, p).max() < 1e-12
        M = J2 @ J1
        assert np.abs(M - np.eye(5)).max() < 1e-12 + 1e-9 * abs(p[4])


def test_rotation_jacobian_finite_difference():
    """Rotate then propagate back to the nominal new x: its derivative is the
    rotation Jacobian (central differences)."""
    P = _params()
    da = 2 * math.pi / 18
    p = np.array([12.0, 40.0, 0.2, 0.5, 0.8])
    x = 300.0
    ok, p1, _, x1, J = O.rotate(P, p, None, x, da)

    def F(q):
        ok, r, _, xr, _ = O.rotate(P, q, None, x, da)
        ok2, r2, _, _, _ = O.propagate(P, r, None, xr, x1)
        return r2

    h = np.array([1e-4, 1e-4, 1e-6, 1e-6, 1e-6])
    Jn = np.zeros((5, 5))
    for j in range(5):
        e = np.zeros(5)
        e[j] = h[j]
        Jn[:, j] = (F(p + e) - F(p - e)) / (2 * h[j])
    assert np.abs(J - Jn).max() < 1e-7


def test_transport_monte_carlo():
    """Sample covariance of propagated states equals J C J^T."""
    P = _params()
    rng = np.random.default_rng(21)
    p = np.array([5.0, 30.0, 0.25, 0.3, -1.2])
    Cm = np.diag([0.05, 0.08, 4e-6, 3e-6, 2.5e-5])
    Cm[0, 2] = Cm[2, 0] = 0.3 * math.sqrt(0.05 * 4e-6)
    Cm[2, 4] = Cm[4, 2] = -0.2 * math.sqrt(4e-6 * 2.5e-5)
    ok, _, Cpred, _, _ = O.propagate(P, p, O.pack(Cm), 250.0, 320.0)
    Cpred = O.unpack(Cpred)
    N = 40000
    L = np.linalg.cholesky(Cm)
    S = p[:, None] + L @ rng.standard_normal((5, N))
    out = np.zeros((5, N))
    for i in range(N):
        ok, q, _, _, _ = O.propagate(P, S[:, i], None, 250.0, 320.0)
        assert ok
        out[:, i] = q
    Cs = np.cov(out)
    sc = np.sqrt(np.outer(np.diag(Cpred), np.diag(Cpred)))
    assert (np.abs(Cs - Cpred) / sc).max() < 5 * math.sqrt(2.0 / N) * 2


def test_highland_value():
    gold = GOLD["highland_theta0_p1_beta1_x0.03"]
    P = _params(mass=0.0, x_over_x0=0.03)
    p = np.array([0.0, 0.0, 0.0, 0.0, 1.0])          # p = 1 GeV/c, normal incidence
    c = O.add_ms(P, p, np.zeros(15))
    th0 = math.sqrt(O.unpack(c)[2, 2])
    assert abs(th0 - gold["value"]) / gold["value"] < gold["rel_tol"]
    M = O.unpack(c)
    assert M[0, 0] == 0 and M[1, 1] == 0 and M[4, 4] == 0


def test_ms_matches_angle_kick_model():
    """Q equals the covariance of (snp, tgl, q/pT) under random angle kicks
    (phi += theta1/cos(lambda), lambda += theta2, |p| fixed)."""
    P = _params()
    rng = np.random.default_rng(4)
    s, t, c = 0.35, 0.6, -0.8
    p = np.array([0.0, 0.0, s, t, c])
    Q = O.unpack(O.add_ms(P, p, np.zeros(15)))
    th0 = math.sqrt(Q[3, 3]) / (1 + t * t)   # theta0 from Q_tt
    N = 400000
    phi = math.asin(s) + rng.standard_normal(N) * th0 / math.cos(math.atan(t))
    lam = math.atan(t) + rng.standard_normal(N) * th0
    pabs = math.sqrt(1 + t * t) / abs(c)
    samp = np.stack([np.sin(phi), np.tan(lam), np.sign(c) / (pabs * np.cos(lam))])
    Cs = np.cov(samp)
    sc = np.sqrt(np.outer(np.diag(Q[2:, 2:]), np.diag(Q[2:, 2:])))
    assert (np.abs(Cs - Q[2:, 2:]) / sc).max() < 0.02
    # theta0 itself: Highland at this momentum and path length
    beta = pabs / math.sqrt(pabs ** 2 + P["mass"] ** 2)
    xi = 0.03 * math.sqrt(1 + t * t) / math.sqrt(1 - s * s)
    assert abs(th0 - 0.0136 / (beta * pabs) * math.sqrt(xi) * (1 + 0.038 * math.log(xi))) < 1e-12


def _rand_spd(rng):
    A = rng.standard_normal((5, 5)) * np.array([0.3, 0.5, 2e-3, 1e-3, 0.05])[:, None]
    return A @ A.T + np.diag([0.01, 0.02, 1e-6, 1e-6, 1e-4])


def test_update_identities():
    rng = np.random.default_rng(9)
    for _ in range(30):
        Cm = _rand_spd(rng)
        p = rng.standard_normal(5)
        tau = rng.choice([0.0, math.tan(math.radians(2)), -math.tan(math.radians(2))])
        vy, vz = 0.04 ** 2, 64 / 12
        ry, rz = rng.standard_normal() * 0.1, rng.standard_normal() * 2
        p2, c2 = O.update(p, O.pack(Cm), ry, rz, tau, vy, vz)
        H = np.array([[1, tau, 0, 0, 0], [0, 1, 0, 0, 0.0]])
        V = np.diag([vy, vz])
        # information form
        Cinf = np.linalg.inv(np.linalg.inv(Cm) + H.T @ np.linalg.inv(V) @ H)
        sc = np.sqrt(np.outer(np.diag(Cinf), np.diag(Cinf)))
        assert (np.abs(O.unpack(c2) - Cinf) / sc).max() < 1e-9
        # gain form p + C H^T (H C H^T + V)^-1 r
        K = Cm @ H.T @ np.linalg.inv(H @ Cm @ H.T + V)
        assert np.abs(p2 - (p + K @ np.array([ry, rz]))).max() < 1e-10 * (1 + np.abs(p2).max())
        assert O.ldl_pd(c2)


def test_update_limits():
    Cm = np.diag([0.5, 3.0, 1e-5, 1e-5, 1e-3])
    p = np.array([1.0, 2.0, 0.1, 0.2, 0.5])
    # V -> 0 pins (y, z) to the measurement (tau = 0: m = (y + ry, z + rz))
    p2, c2 = O.update(p, O.pack(Cm), 0.3, -0.7, 0.0, 1e-20, 1e-20)
    assert abs(p2[0] - 1.3) < 1e-12 and abs(p2[1] - 1.3) < 1e-12
    # V -> infinity changes nothing
    p3, c3 = O.update(p, O.pack(Cm), 0.3, -0.7, 0.0, 1e30, 1e30)
    assert np.abs(p3 - p).max() < 1e-20 + 1e-12 and np.abs(O.unpack(c3) - Cm).max() < 1e-12
    # diagonal C, no tilt: inverse-variance weighted mean in y
    p4, c4 = O.update(p, O.pack(Cm), 0.3, 0.0, 0.0, 0.25, 1.0)
    ymeas = 1.3
    wm = (1.0 / 0.5 + ymeas / 0.25) / (1 / 0.5 + 1 / 0.25)
    assert abs(p4[0] - wm) < 1e-13
    assert abs(O.unpack(c4)[0, 0] - 1 / (1 / 0.5 + 1 / 0.25)) < 1e-13


def test_ldl_detects_indefinite():
    assert O.ldl_pd(O.pack(np.eye(5)))
    M = np.eye(5)
    M[0, 1] = M[1, 0] = 1.0000001
    assert not O.ldl_pd(O.pack(M))
    assert not O.ldl_pd(O.pack(np.diag([1, 1, 0, 1, 1.0])))
