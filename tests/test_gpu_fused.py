"""trd_load_and_match (binning and the seeds' ordering on two streams,
joined before the match) against trd_load_tracklets + trd_match: results
and binning bit-identical, alone and replayed from a captured graph."""
import numpy as np
import pytest

from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _frames():
    return synth.generate_frames(11, 6, [1500, 300, 2500, 1, 900, 2000], [0.5] * 6,
                                 params_over=dict(y_bin_w=8.0, n_yb=16), ineff_frac=0.1)


def _np(out):
    return {k: v.cpu().numpy() for k, v in out.items() if v is not None}


def _separate(w, d, prec, flags=0, n_hyp=0):
    P = dict(w["params"], **({"n_hyp": n_hyp, "chi2_penalty": 9.0} if n_hyp else {}))
    m = B.Matcher(P, prec, flags=flags)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    out = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    torch.cuda.synchronize()
    off, srt = m.binning()
    torch.cuda.synchronize()
    r = _np(out)
    r["offsets"], r["sorted"] = off.cpu().numpy(), srt.cpu().numpy()
    m.close()
    return r


def _fused(w, d, prec, flags=0, n_hyp=0):
    P = dict(w["params"], **({"n_hyp": n_hyp, "chi2_penalty": 9.0} if n_hyp else {}))
    m = B.Matcher(P, prec, flags=flags)
    out = m.load_and_match(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"], d["p"], d["cov"],
                           d["x"], d["sector"], tgroup=d["group"])
    torch.cuda.synchronize()
    off, srt = m.binning()
    torch.cuda.synchronize()
    r = _np(out)
    r["offsets"], r["sorted"] = off.cpu().numpy(), srt.cpu().numpy()
    m.close()
    return r


def _same(a, b):
    assert a.keys() == b.keys()
    for k in a:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


@pytest.mark.parametrize("prec", ["fp32", "fp64", "fp32_cov64"])
def test_fused_equals_load_then_match(prec):
    w = _frames()
    d = B.device_inputs(synth.to_device_layout(w), prec)
    _same(_fused(w, d, prec), _separate(w, d, prec))


@pytest.mark.parametrize("flags,n_hyp", [(B.TRD_CFG_INPUT_ORDER, 0), (B.TRD_CFG_PERSISTENT, 0), (0, 2)])
def test_fused_equals_load_then_match_other_launches(flags, n_hyp):
    """Caller's order (no fork), the persistent grid, two hypotheses."""
    w = _frames()
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    _same(_fused(w, d, "fp32", flags, n_hyp), _separate(w, d, "fp32", flags, n_hyp))


def test_fused_without_tracks_or_tracklets():
    w = _frames()
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    m = B.Matcher(w["params"], "fp32")
    # no tracks: only the binning
    e = d["x"][:0]
    m.load_and_match(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"], d["p"][:, :0].contiguous(),
                     d["cov"][:, :0].contiguous(), e, d["sector"][:0], tgroup=d["group"][:0])
    torch.cuda.synchronize()
    off, _ = m.binning()
    ref = _separate(w, d, "fp32")
    assert np.array_equal(off.cpu().numpy(), ref["offsets"])
    # no tracklets: every track unmatched
    y0 = d["y"][:0]
    out = m.load_and_match(y0, d["z"][:0], d["dy"][:0], d["det_row"][:0], d["tgroup"][:0], w["n_groups"], d["p"],
                           d["cov"], d["x"], d["sector"], tgroup=d["group"])
    torch.cuda.synchronize()
    assert int(out["n_match"].max().item()) == 0
    assert int((out["idx"] >= 0).sum().item()) == 0
    m.close()


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fused_graph_replays_equal_eager(prec):
    """The fork onto the context's stream and the join, captured: three
    replays with eager work of another context between them."""
    w = _frames()
    d = B.device_inputs(synth.to_device_layout(w), prec)
    n = w["n_tracks"]
    ref = _separate(w, d, prec)
    m = B.Matcher(w["params"], prec)
    m.reserve(w["n_tracklets"], w["n_groups"], n)
    out = m.alloc_results(n)

    def body():
        m.load_and_match(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"], d["p"], d["cov"],
                         d["x"], d["sector"], tgroup=d["group"], out=out)

    stream = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        body()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        body()
    torch.cuda.synchronize()
    other = B.Matcher(w["params"], prec)
    for rep in range(3):
        for v in out.values():
            if v is not None:
                v.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        got = _np(out)
        for k in got:
            assert np.array_equal(got[k], ref[k], equal_nan=True), (rep, k)
        other.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
        o2 = other.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
        torch.cuda.synchronize()
        assert np.array_equal(o2["idx"].cpu().numpy(), ref["idx"])
    other.close()
    m.close()
