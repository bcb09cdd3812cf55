"""Inclination-dependent tracklet resolutions and the Lorentz-angle offset of
the deflection on the GPU, against the FP64 oracle (Sect. 3 and Fig. 3: the
y and dy widths are second-order polynomials in sin(phi) evaluated for every
candidate, smallest at the Lorentz angle, about 8 degrees at 0.5 T).

The workloads draw each tracklet's noise at the true inclination and offset
its deflection by L tan(psi_L); the matcher evaluates the polynomials at its
predicted sin(phi), in the road, the dy gate and the update.  Element by
element through the C ABI in all three precisions, with a bound on the
flagged share.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu
from tests.test_gpu_parity import check_binning, run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_cache = {}


def _wl(key):
    if key not in _cache:
        params = dict(synth.inclined_resolution())
        if key == "c2":
            _cache[key] = synth.generate("c2_frame_20k", params=params)
        else:
            params.update(y_bin_w=4.0, n_yb=32, tilt=synth.tilt_pm2deg(),
                          dx_chamber=np.random.default_rng(71).uniform(-0.5, 0.5, 540))
            _cache[key] = synth.generate(n_tracks=3000, seed=73, fake_ratio=0.5, ineff_frac=0.1,
                                         params=params)
    return _cache[key]


def test_workload_has_non_zero_slope_curvature_and_offset():
    P = _wl("c2")["params"]
    assert P["sigma_y"][1] != 0 and P["sigma_y"][2] != 0
    assert P["sigma_dy"][1] != 0 and P["sigma_dy"][2] != 0
    assert abs(P["tan_psi"] - np.tan(np.radians(8.0))) < 1e-15


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_frame_20k_inclined_resolution(prec):
    w = _wl("c2")
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, res, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()
    # with the offset, true tracklets pass the dy gate: most layers match
    assert (res["idx"] >= 0).sum() > 0.5 * 6 * w["n_tracks"]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tilted_misaligned_inclined_resolution(prec):
    w = _wl("tilt")
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, res, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_constant_widths_change_the_decisions():
    """Sensitivity: the same workload matched with the polynomials' constant
    terms only (and no offset) gives other indices on the GPU, so the
    parity above exercises the slope, curvature and offset terms."""
    w = _wl("c2")
    a = run_gpu(w, "fp64")
    P0 = dict(w["params"])
    P0["sigma_y"] = [P0["sigma_y"][0], 0.0, 0.0]
    P0["sigma_dy"] = [P0["sigma_dy"][0], 0.0, 0.0]
    P0["tan_psi"] = 0.0
    b = run_gpu(w, "fp64", params=P0)
    changed = np.any(a["idx"] != b["idx"], axis=0).mean()
    assert changed > 0.05, changed
