"""Field inhomogeneity on the GPU against the FP64 oracle (Sect. 3: the
precise extrapolation accounts for the field; synthetic map Bz(r, z) = Bz0
(1 + b_r (r/370)^2 + b_z (z/360)^2) with b_r = -0.02, b_z = -0.04).

The workload's tracks and tracklets are simulated in that field (the
generator integrates the equation of motion in the global frame); matching
and the TRD-only refit integrate it with the Runge-Kutta step of the
configuration, element by element through the C ABI, in all three
precisions, with tilted pads and misaligned chambers in one case.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu
from tests.test_gpu_parity import check_binning, run_gpu
from tests.test_gpu_refit import compare as refit_compare
from tests.test_gpu_refit import gpu_match_refit

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_cache = {}


def _wl(key):
    if key not in _cache:
        params = dict(synth.field_map_overrides(), y_bin_w=8.0, n_yb=16)
        if key == "tilt":
            params.update(tilt=synth.tilt_pm2deg(), dx_chamber=np.random.default_rng(81).uniform(-0.5, 0.5, 540))
        _cache[key] = synth.generate(n_tracks=3000, seed=83 if key == "tilt" else 82, fake_ratio=0.5,
                                     ineff_frac=0.1, params=params)
    return _cache[key]


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_field_map_frame(prec):
    w = _wl("plain")
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, res, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()
    assert (res["idx"] >= 0).sum() > 0.5 * 6 * w["n_tracks"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_field_map_tilted_misaligned(prec):
    w = _wl("tilt")
    res = run_gpu(w, prec)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    tol = pu.tilted_float_tol(w["params"]) if prec != "fp64" else None
    rep = pu.compare(ref, res, prec, state_tol_max=tol, q999_tol=tol)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_the_map_changes_the_answer():
    """The map is applied on the GPU: the same tracks matched as if the field
    were uniform end with other states."""
    w = _wl("plain")
    a = run_gpu(w, "fp64")
    U = dict(w["params"], field_br=0.0, field_bz=0.0)
    b = run_gpu(w, "fp64", params=U)
    ok = (a["status"] == 0) & (b["status"] == 0) & (a["n_match"] == 6) & (b["n_match"] == 6)
    assert np.median(np.abs(a["p"][0, ok] - b["p"][0, ok])) > 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_refit_in_the_field_map(prec):
    w = _wl("plain")
    matched, got = gpu_match_refit(w, prec)
    ref = O.refit(w["params"], matched, matched["idx"], w)
    print(refit_compare(ref, got, prec))
