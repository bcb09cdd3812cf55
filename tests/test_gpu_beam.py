"""Several hypotheses per track (Sect. 3, Fig. 2) on the HIP path against the
FP64 oracle's multi-hypothesis matcher, through the C ABI."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_cache = {}


def workload(name):
    if name not in _cache:
        _cache[name] = synth.generate(name)
    return _cache[name]


def beam_params(P, n_hyp, penalty=None):
    Q = dict(P)
    Q["n_hyp"] = n_hyp
    Q["chi2_penalty"] = P["chi2_max"] if penalty is None else penalty
    return Q


def run(w, P, prec, flags=0):
    d = B.device_inputs(synth.to_device_layout(w), prec)
    m = B.Matcher(P, prec, flags=flags)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    out = pu.to_numpy(m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"]))
    torch.cuda.synchronize()
    m.close()
    return out


@pytest.mark.parametrize("n_hyp", [1, 2, 4, 8])
@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_small_frame(prec, n_hyp):
    w = workload("c1_small_fp64")
    P = beam_params(w["params"], n_hyp, penalty=None if n_hyp == 1 else 9.0)
    got = run(w, P, prec)
    ref = O.match(P, w, threads=0, margins=pu.BEAM_MARGINS[prec])
    rep = pu.compare(ref, got, prec, max_flag_share=pu.MAX_FLAG_SHARE_BEAM)
    print(rep.summary())
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_frame_20k_four_hypotheses(prec):
    w = workload("c2_frame_20k")
    P = beam_params(w["params"], 4, penalty=9.0)
    got = run(w, P, prec)
    sel = np.arange(0, w["n_tracks"], 4)
    ref = O.match(P, w, threads=0, margins=pu.BEAM_MARGINS[prec], track_slice=sel)
    rep = pu.compare(ref, got, prec, sel=sel, max_flag_share=pu.MAX_FLAG_SHARE_BEAM)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_distortion_batch_sampled():
    """The 450k distortion batch with four hypotheses (float path), 1,500
    sampled tracks against the oracle."""
    w = synth.generate("c5_distortion_450k")
    P = beam_params(w["params"], 4, penalty=9.0)
    got = run(w, P, "fp32")
    sel = np.sort(np.random.default_rng(11).choice(w["n_tracks"], 1500, replace=False))
    ref = O.match(P, w, threads=0, margins=pu.BEAM_MARGINS["fp32"], track_slice=sel)
    rep = pu.compare(ref, got, "fp32", sel=sel, max_flag_share=pu.MAX_FLAG_SHARE_BEAM_WIDE)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_forced_fallback_equals_double_covariance_beam():
    w = workload("c1_small_fp64")
    P = beam_params(w["params"], 4, penalty=9.0)
    a = run(w, P, "fp32", flags=B.TRD_CFG_FORCE_FALLBACK)
    b = run(w, P, "fp32_cov64")
    assert np.all(a["status"] & B.TRK_FP64_FALLBACK)
    assert np.array_equal(a["status"] & ~B.TRK_FP64_FALLBACK, b["status"])
    for k in ("idx", "p", "cov", "x", "sector", "chi2", "n_match"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_zero_penalty_takes_no_tracklets():
    w = workload("c1_small_fp64")
    got = run(w, beam_params(w["params"], 2, penalty=0.0), "fp32")
    assert np.all(got["n_match"] == 0) and np.all(got["idx"] == -1)
