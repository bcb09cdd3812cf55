"""Bin + match captured as one HIP graph (multi-frame batches) and the
launch-shape autotuner, against eager runs and the FP64 oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu
from tests.test_gpu_parity import run_gpu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _snapshot(out):
    return {k: (v.clone() if v is not None else None) for k, v in out.items()}


def _capture(m, d, n_groups, out):
    stream = torch.cuda.current_stream()

    def body():
        m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], n_groups)
        m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)

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
    return g


@pytest.mark.parametrize("prec,flags", [("fp32", 0), ("fp64", 0), ("fp32", B.TRD_CFG_PERSISTENT)])
def test_graph_replays_equal_eager(prec, flags):
    w = synth.generate_frames(5, 8, [1500, 300, 2500, 1, 900, 2000, 1200, 700],
                              [0.5] * 8, params_over=dict(y_bin_w=8.0, n_yb=16), ineff_frac=0.1)
    d = B.device_inputs(synth.to_device_layout(w), prec)
    n = w["n_tracks"]
    m = B.Matcher(w["params"], prec, flags=flags)
    m.reserve(w["n_tracklets"], w["n_groups"], n)
    out = m.alloc_results(n)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)
    torch.cuda.synchronize()
    eager = {k: v.cpu().numpy() for k, v in _snapshot(out).items() if v is not None}
    g = _capture(m, d, w["n_groups"], out)
    other = B.Matcher(w["params"], prec)
    for rep in range(3):
        for v in out.values():
            if v is not None:
                v.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        for k in eager:
            assert np.array_equal(got[k], eager[k], equal_nan=True), (rep, k)
        # unrelated eager work on the same device between replays
        other.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
        o2 = other.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
        torch.cuda.synchronize()
        assert np.array_equal(o2["idx"].cpu().numpy(), eager["idx"])
    other.close()
    m.close()


def test_graph_of_a_timed_matcher():
    """A matcher that times its match kernel (TRD_CFG_TIME_KERNEL) is timed by
    the kernel's own dispatch when eager and can still be captured (its events
    are then recorded around the kernel); replays give the eager results."""
    w = synth.generate("c2_frame_20k")
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    n = w["n_tracks"]
    m = B.Matcher(w["params"], "fp32", flags=B.TRD_CFG_TIME_KERNEL)
    m.reserve(w["n_tracklets"], w["n_groups"], n)
    out = m.alloc_results(n)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)
    torch.cuda.synchronize()
    t = m.kernel_times()
    assert len(t) == 1 and 0.0 < t[0] < 100.0, t
    eager = {k: v.cpu().numpy() for k, v in _snapshot(out).items() if v is not None}
    g = _capture(m, d, w["n_groups"], out)
    for rep in range(3):
        for v in out.values():
            if v is not None:
                v.fill_(-7)
        g.replay()
        torch.cuda.synchronize()
        got = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
        for k in eager:
            assert np.array_equal(got[k], eager[k], equal_nan=True), (rep, k)
    m.close()


def test_multiframe_batch_graph_full_size_sampled():
    """64 frames (~1.4M tracks, ~12M tracklets) replayed as one graph, float
    path; 2,000 sampled tracks against the oracle, group isolation in full."""
    w = synth.multiframe_64()
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    n = w["n_tracks"]
    m = B.Matcher(w["params"], "fp32")
    m.reserve(w["n_tracklets"], w["n_groups"], n)
    out = m.alloc_results(n)
    g = _capture(m, d, w["n_groups"], out)
    g.replay()
    torch.cuda.synchronize()
    res = pu.to_numpy(out)
    m.close()
    sel = np.sort(np.random.default_rng(3).choice(n, 2000, replace=False))
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"], track_slice=sel)
    rep = pu.compare(ref, res, "fp32", sel=sel)
    print(rep.summary())
    assert rep.ok, rep.summary()
    idx = res["idx"]
    mk = idx >= 0
    assert np.array_equal(w["tkl_group"][idx[mk]], np.broadcast_to(w["group"], idx.shape)[mk])


def test_autotune_picks_a_listed_shape_and_geometry(tmp_path):
    """The tuner times the listed cell geometries, then the launch shapes
    (and the persistent grid with one lane per track) with the best one; its
    choice gives results bit-identical to the workload's own geometry (the
    search does not depend on the bins); the cache returns the same record."""
    from paper_2003_03174_amd import autotune
    w = synth.generate("c2_frame_20k")
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    geos = [dict(y_bin_w=4.0, n_yb=32, dy_bin_w=0.0625, n_db=1), dict(y_bin_w=16.0, n_yb=8, dy_bin_w=0.0625, n_db=1)]
    r = autotune.tune(w["params"], d, 1, "fp32", shapes=((256, 1), (256, 8), (128, 4)), reps=2,
                      cache_path=str(tmp_path / "c.json"), geometries=geos)
    assert (r["block_size"], r["search_lanes"]) in {(256, 1), (256, 8), (128, 4)}
    assert len(r["table"]) == 4 and all(t[3] > 0 for t in r["table"])
    assert len(r["bin_table"]) == 3 and r["bins"] in geos + [dict(y_bin_w=8.0, n_yb=16, dy_bin_w=0.0625, n_db=1)]
    r2 = autotune.tune(w["params"], d, 1, "fp32", cache_path=str(tmp_path / "c.json"))
    assert r2["table"] == [list(t) for t in r["table"]] or r2["table"] == r["table"]
    base = run_gpu(w, "fp32")
    for gq in geos:
        o = run_gpu(w, "fp32", params=dict(w["params"], **gq))
        for k in ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status"):
            assert np.array_equal(o[k], base[k], equal_nan=True), (gq, k)
