"""HIP path vs the FP64 oracle, element by element, through the C ABI.

Sizes: 1,000-track and 20,000-track frames (several workgroups, ragged tails),
multi-frame batches, and the full 450,000-track distortion batch in the
launch configuration the benchmark times (sampled tracks against the
oracle, binning compared in full).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

_cache = {}


def workload(name, **kw):
    key = (name, tuple(sorted((k, str(v)) for k, v in kw.items())))
    if key not in _cache:
        _cache[key] = synth.generate(name, **kw) if name else synth.generate(**kw)
    return _cache[key]


def run_gpu(w, prec, block_size=0, params=None, search_lanes=0, flags=0, groups=True):
    """groups=False passes no group arrays (every tracklet and seed in group 0)."""
    P = params or w["params"]
    lay = synth.to_device_layout(w)
    d = B.device_inputs(lay, prec)
    m = B.Matcher(P, prec, block_size=block_size, search_lanes=search_lanes, flags=flags)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"] if groups else None, w["n_groups"])
    out = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"] if groups else None)
    torch.cuda.synchronize()
    res = pu.to_numpy(out)
    off, srt = m.binning()
    torch.cuda.synchronize()
    res["offsets"] = off.cpu().numpy().view(np.uint32)
    res["sorted"] = srt.cpu().numpy()
    m.close()
    return res


def check_binning(w, res):
    perm, off = O.bin_tracklets(w["params"], w)
    assert np.array_equal(res["offsets"], off), "cell offsets differ"
    nv = int(off[-1])
    srt = res["sorted"][:nv]
    gidx = srt[:, 3].copy().view(np.int32)
    assert np.array_equal(gidx, perm[:nv]), "sorted permutation differs"
    assert np.array_equal(srt[:, 0], w["tkl_y"][gidx].astype(np.float32))
    assert np.array_equal(srt[:, 1], w["tkl_dy"][gidx].astype(np.float32))
    assert np.array_equal(srt[:, 2], w["tkl_z"][gidx].astype(np.float32))


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_small_frame(prec):
    w = workload("c1_small_fp64")
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, res, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_tilted_pads_and_misaligned_chambers(prec):
    rng = np.random.default_rng(7)
    params = dict(y_bin_w=4.0, n_yb=32, tilt=synth.tilt_pm2deg(), dx_chamber=rng.uniform(-0.5, 0.5, 540))
    w = workload(None, n_tracks=3000, seed=17, fake_ratio=0.5, ineff_frac=0.1, params=params)
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, res, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
@pytest.mark.parametrize("tilt", [False, True])
def test_deflection_bins(prec, tilt):
    """Cells split in dy as well (y bins innermost): binning bit-exact, parity."""
    params = dict(y_bin_w=8.0, n_yb=16, dy_bin_w=0.125, n_db=64)
    if tilt:
        params["tilt"] = synth.tilt_pm2deg()
        params["dx_chamber"] = np.random.default_rng(9).uniform(-0.5, 0.5, 540)
    w = workload(None, n_tracks=4000, seed=29, fake_ratio=0.5, ineff_frac=0.1, pt_dist="pow3",
                 params=params)
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    # Float state with tilted pads: the bound of pu.tilted_float_tol (the
    # float y's unit roundoff carried into z by the update's tilt gain)
    tol = pu.tilted_float_tol(w["params"]) if (tilt and prec != "fp64") else None
    rep = pu.compare(ref, res, prec, state_tol_max=tol, q999_tol=tol)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_cells_per_chamber_above_one_chunk():
    """More cells per chamber (4 cm y bins x 1/8 cm dy bins x 18 rows) than
    the cell sort orders in one LDS chunk: binning bit-exact, parity."""
    params = dict(y_bin_w=4.0, n_yb=32, dy_bin_w=0.125, n_db=64)
    w = workload(None, n_tracks=3000, seed=31, fake_ratio=0.5, ineff_frac=0.1, params=params)
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()


def test_unaligned_tracklet_arrays():
    """Tracklet arrays at an offset of one element (not 16-byte aligned):
    binning bit-exact, parity."""
    w = workload("c1_small_fp64")
    lay = synth.to_device_layout(w)
    d = B.device_inputs(lay, "fp32")
    m = B.Matcher(w["params"], "fp32")
    shifted = {}
    for k in ("y", "z", "dy", "det_row", "tgroup"):
        buf = torch.empty(d[k].numel() + 1, dtype=d[k].dtype, device=d[k].device)
        buf[1:].copy_(d[k])
        shifted[k] = buf[1:]
    assert shifted["y"].data_ptr() % 16 != 0
    m.load(shifted["y"], shifted["z"], shifted["dy"], shifted["det_row"], shifted["tgroup"], w["n_groups"])
    out = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    torch.cuda.synchronize()
    res = pu.to_numpy(out)
    off, srt = m.binning()
    torch.cuda.synchronize()
    res["offsets"] = off.cpu().numpy().view(np.uint32)
    res["sorted"] = srt.cpu().numpy()
    m.close()
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()


def test_cells_per_bucket_above_one_chunk():
    """A chamber of 1 cm y bins x 1/16 cm dy bins x 18 rows (294912 cells):
    the cell sort goes over 18 LDS chunks: binning bit-exact, parity."""
    params = dict(y_bin_w=1.0, n_yb=128, dy_bin_w=0.0625, n_db=128)
    w = workload(None, n_tracks=1500, seed=37, fake_ratio=0.5, ineff_frac=0.1, params=params)
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_frame_20k(prec):
    w = workload("c2_frame_20k")
    res = run_gpu(w, prec)
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, res, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_multi_frame_groups():
    w = synth.generate_frames(2, 6, [500, 3000, 1, 2500, 800, 1200], [0.2, 0.8, 0.5, 0.3, 0.6, 0.4],
                              params_over=dict(y_bin_w=8.0, n_yb=16), ineff_frac=0.1)
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()
    m = res["idx"] >= 0
    assert np.array_equal(w["tkl_group"][res["idx"][m]], np.broadcast_to(w["group"], m.shape)[m])


def test_multi_frame_groups_with_deflection_bins():
    """Five groups of 540 chambers with 36 deflection bins: chambers too large
    to be sorted together, so the partition by chamber takes two passes
    (an 11-bit digit, then an 8-bit one).  Binning bit-exact, parity."""
    w = synth.generate_frames(4, 5, [900, 1, 2000, 400, 1500], [0.5, 0.2, 0.7, 0.4, 0.6],
                              params_over=dict(y_bin_w=8.0, n_yb=16, dy_bin_w=0.25, n_db=36),
                              ineff_frac=0.1)
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()


def test_distortion_batch_full_size_sampled():
    """450k tracks / ~3.8M tracklets, float path with block 256 as timed:
    binning bit-exact in full, 3000 sampled tracks against the oracle."""
    w = workload("c5_distortion_450k")
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    sel = np.random.default_rng(0).choice(w["n_tracks"], 3000, replace=False)
    sel.sort()
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"], track_slice=sel)
    rep = pu.compare(ref, res, "fp32", sel=sel)
    print(rep.summary())
    assert rep.ok, rep.summary()
    # whole-batch properties: every match is a tracklet of the right layer/sector
    idx = res["idx"]
    m = idx >= 0
    lay = np.broadcast_to(np.arange(6)[:, None], idx.shape)
    assert np.array_equal(w["tkl_layer"][idx[m]], lay[m])


def test_fp32_cov64_full_size_sampled():
    """The float state with a double covariance on the whole 450k batch."""
    w = workload("c5_distortion_450k")
    res = run_gpu(w, "fp32_cov64")
    sel = np.random.default_rng(2).choice(w["n_tracks"], 1500, replace=False)
    sel.sort()
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32_cov64"], track_slice=sel)
    rep = pu.compare(ref, res, "fp32_cov64", sel=sel)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_fp64_full_size_sampled():
    w = workload("c5_distortion_450k")
    res = run_gpu(w, "fp64")
    sel = np.random.default_rng(1).choice(w["n_tracks"], 1500, replace=False)
    sel.sort()
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp64"], track_slice=sel)
    rep = pu.compare(ref, res, "fp64", sel=sel)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_forced_fallback_equals_double_covariance_path():
    """Test hook: every track takes the re-run; the result must be bit-identical
    to the float-state / double-covariance path (same arithmetic)."""
    w = workload("c2_frame_20k")
    P = w["params"]
    lay = synth.to_device_layout(w)
    d = B.device_inputs(lay, "fp32")
    outs = []
    for prec, flags in (("fp32", B.TRD_CFG_FORCE_FALLBACK), ("fp32_cov64", 0)):
        m = B.Matcher(P, prec, flags=flags)
        m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
        outs.append(pu.to_numpy(m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])))
        torch.cuda.synchronize()
        m.close()
    a, b = outs
    assert np.all(a["status"] & B.TRK_FP64_FALLBACK)
    assert np.array_equal(a["status"] & ~B.TRK_FP64_FALLBACK, b["status"])
    for k in ("idx", "p", "cov", "x", "sector", "chi2", "n_match"):
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_fallback_for_seeds_singular_in_float():
    """Seeds whose y-z covariance block [[3, 1], [1, fl32(1/3)]] is positive
    definite in double but singular in float: the float path must hand them to
    the double-covariance re-run, whose result agrees with the oracle."""
    w = dict(workload("c1_small_fp64"))
    w["cov"] = w["cov"].copy()
    sel = np.arange(0, w["n_tracks"], 10)
    w["cov"][0, sel] = 3.0
    w["cov"][1, sel] = 1.0
    w["cov"][5, sel] = float(np.float32(1.0 / 3.0))
    assert O.ldl_pd(w["cov"][:, sel[0]])
    res = run_gpu(w, "fp32")
    st = res["status"].astype(np.int64)
    fb = np.nonzero((st & B.TRK_FP64_FALLBACK) != 0)[0]
    assert set(fb.tolist()) == set(sel.tolist()), (fb.size, sel.size)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32_cov64"])
    rep = pu.compare(ref, res, "fp32_cov64")
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_empty_and_single():
    w = workload("c1_small_fp64")
    w0 = dict(w)
    for k in ("tkl_y", "tkl_z", "tkl_dy"):
        w0[k] = np.zeros(0)
    w0["tkl_det_row"] = np.zeros(0, np.uint32)
    w0["tkl_group"] = np.zeros(0, np.int32)
    res = run_gpu(w0, "fp32")
    assert np.all(res["idx"] == -1) and np.all(res["n_match"] == 0)
    ref = O.match(w0["params"], w0, threads=0, margins=pu.MARGINS["fp32"])
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()
    w1 = dict(w)
    for k in ("p", "cov"):
        w1[k] = np.ascontiguousarray(w[k][:, 5:6])
    for k in ("x", "sector", "group"):
        w1[k] = np.ascontiguousarray(w[k][5:6])
    w1["n_tracks"] = 1
    res = run_gpu(w1, "fp64")
    ref = O.match(w1["params"], w1, threads=0, margins=pu.MARGINS["fp64"])
    # one track: the share bound is no statement here (a flagged track is
    # still compared on the layers before its flag)
    assert pu.compare(ref, res, "fp64", max_flag_share=1.0).ok


def test_invalid_tracklets_and_bad_seeds():
    w = dict(workload("c1_small_fp64"))
    w["tkl_det_row"] = w["tkl_det_row"].copy()
    w["tkl_y"] = w["tkl_y"].copy()
    w["tkl_det_row"][3] = (541 << 5) | 2
    w["tkl_det_row"][4] = (10 << 5) | 25
    w["tkl_y"][5] = np.nan
    w["p"] = w["p"].copy()
    w["sector"] = w["sector"].copy()
    w["p"][0, 0] = np.nan
    w["sector"][1] = 99
    w["p"][2, 2] = float(np.float32(0.97))
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    assert res["offsets"][-1] == w["n_tracklets"] - 3
    st = res["status"]
    for i in (0, 1, 2):
        assert st[i] & B.TRK_BAD_INPUT and res["n_match"][i] == 0
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    assert np.all(ref["status"][:3] == B.TRK_BAD_INPUT)
    rep = pu.compare(ref, res, "fp32")
    assert rep.ok, rep.summary()


def _with_edge_values(w):
    """Tracklets and seeds at the edges of the cell key's and the seeds'
    order key's domains."""
    w = dict(w)
    for k in ("tkl_y", "tkl_z", "tkl_dy", "tkl_det_row", "tkl_group", "p", "sector", "group"):
        w[k] = w[k].copy()
    y, z, dy, dr, tg = w["tkl_y"], w["tkl_z"], w["tkl_dy"], w["tkl_det_row"], w["tkl_group"]
    # non-finite: dropped; finite far outside the bins' span: the outer bins
    y[0], y[1], y[2], y[3] = np.inf, -np.inf, 1e30, -1e30
    z[4], z[5] = np.nan, np.inf
    dy[6], dy[7], dy[8], dy[9] = np.nan, -np.inf, 1e30, -1e30
    # the last chamber slot and row (kept); chamber 540 and an all-ones word (dropped)
    dr[10] = (539 << 5) | (w["params"]["n_rows"] - 1)
    dr[11] = 540 << 5
    dr[12] = 0xFFFFFFFF
    ng = w["n_groups"]
    if ng > 1:
        tg[13], tg[14], tg[15] = -1, ng, 1 << 30
    # seeds: non-finite z and q/pT, a sector and (with groups) a group out of
    # range are bad input; y and z beyond the order key's bins are clamped
    p = w["p"]
    p[1, 0] = np.nan
    p[4, 1] = np.inf
    w["sector"][2] = -1
    if ng > 1:
        w["group"][3] = ng
    p[0, 4] = 80.0
    p[0, 5] = -100.0
    p[1, 6] = 600.0
    return w


@pytest.mark.parametrize("grouped", [False, True])
def test_edge_values_of_binning_and_order(grouped):
    """Infinities, NaN, finite values far outside the bins' span, chambers,
    rows and groups out of range, in the tracklets and in the seeds: binning
    bit-exact against the oracle, results against the oracle.  Without
    groups, passing no group arrays gives the binning and results of
    zero-filled ones bit for bit, in separate calls and in the fused one."""
    params = dict(dy_bin_w=0.125, n_db=64)
    if grouped:
        w = synth.generate_frames(43, 3, [700, 500, 900], [0.5, 0.3, 0.7], params_over=params)
    else:
        w = workload(None, n_tracks=2000, seed=41, fake_ratio=0.5, params=params)
    w = _with_edge_values(w)
    res = run_gpu(w, "fp32")
    check_binning(w, res)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS["fp32"])
    bad = (0, 1, 2, 3) if grouped else (0, 1, 2)
    for i in bad:
        assert ref["status"][i] == B.TRK_BAD_INPUT and res["status"][i] & B.TRK_BAD_INPUT, i
    rep = pu.compare(ref, res, "fp32")
    print(rep.summary())
    assert rep.ok, rep.summary()
    if grouped:
        return
    keys = ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status", "offsets", "sorted")
    res0 = run_gpu(w, "fp32", groups=False)
    for k in keys:
        assert np.array_equal(res0[k], res[k], equal_nan=True), k
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    m = B.Matcher(w["params"], "fp32")
    out = m.load_and_match(d["y"], d["z"], d["dy"], d["det_row"], None, 1, d["p"], d["cov"], d["x"],
                           d["sector"], tgroup=None)
    torch.cuda.synchronize()
    fused = pu.to_numpy(out)
    m.close()
    for k in keys[:-2]:
        assert np.array_equal(fused[k], res[k], equal_nan=True), k


def test_deterministic_repeats():
    w = workload("c2_frame_20k")
    a = run_gpu(w, "fp32")
    b = run_gpu(w, "fp32")
    for k in ("idx", "p", "cov", "chi2", "status", "offsets", "sorted"):
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("prec", ["fp32", "fp32_cov64"])
def test_launch_shapes_agree(prec):
    """Block size and lanes per track change the schedule, not the arithmetic:
    results are bit-identical across launch shapes."""
    w = workload("c2_frame_20k")
    base = run_gpu(w, prec, block_size=256, search_lanes=1)
    for bs, lanes in ((64, 4), (128, 8), (256, 16), (192, 32), (256, 64)):
        o = run_gpu(w, prec, block_size=bs, search_lanes=lanes)
        for k in ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status"):
            assert np.array_equal(o[k], base[k], equal_nan=True), (bs, lanes, k)


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_persistent_grid_agrees(prec):
    """The persistent grid (resident workgroups pulling blocks of tracks) runs
    the same per-track arithmetic: bit-identical to the plain launch, also on
    a second call through the same context (work counter cleared)."""
    w = workload("c2_frame_20k")
    base = run_gpu(w, prec, block_size=256, search_lanes=1)
    P = w["params"]
    d = B.device_inputs(synth.to_device_layout(w), prec)
    for bs in (64, 256):
        m = B.Matcher(P, prec, block_size=bs, search_lanes=1, flags=B.TRD_CFG_PERSISTENT)
        m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
        for call in range(2):
            o = pu.to_numpy(m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"]))
            torch.cuda.synchronize()
            for k in ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status"):
                assert np.array_equal(o[k], base[k], equal_nan=True), (bs, call, k)
        m.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_spatial_track_order_is_invisible(prec):
    """The default launch matches the tracks in a spatial order (rows of state
    in, rows of results out); results must be bit-identical to the caller's
    order, here on several frames with rejected seeds and forced re-runs."""
    w = synth.generate_frames(5, 4, [3000, 1, 2500, 900], [0.5] * 4,
                              params_over=dict(y_bin_w=8.0, n_yb=16), ineff_frac=0.1)
    w = dict(w)
    w["p"] = w["p"].copy()
    w["sector"] = w["sector"].copy()
    w["p"][0, 7] = np.nan
    w["sector"][11] = 40
    flags = [0, B.TRD_CFG_FORCE_FALLBACK] if prec == "fp32" else [0]
    for f in flags:
        a = run_gpu(w, prec, flags=f)
        b = run_gpu(w, prec, flags=f | B.TRD_CFG_INPUT_ORDER)
        for k in ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status"):
            assert np.array_equal(a[k], b[k], equal_nan=True), (f, k)
    ref = O.match(w["params"], w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, a, prec)
    assert rep.ok, rep.summary()


def test_kernel_times():
    """TRD_CFG_TIME_KERNEL: one positive duration per match call, oldest
    first, and a fresh count after each read; ESTATE without the flag."""
    w = workload("c1_small_fp64")
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    m = B.Matcher(w["params"], "fp32", flags=B.TRD_CFG_TIME_KERNEL)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    for _ in range(3):
        m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    t = m.kernel_times()
    assert len(t) == 3 and all(v > 0 for v in t)
    assert m.kernel_times() == []
    m.close()
    m = B.Matcher(w["params"], "fp32")
    with pytest.raises(B.TrdError):
        m.kernel_times()
    m.close()


def test_pending_hip_error_is_reported_by_the_next_call():
    """A HIP error left pending on the calling thread (here a failed
    hipSetDevice, which touches no device memory) makes the next call return
    TRD_EDEVICE without enqueuing anything; the error is consumed, so the
    call after it runs normally and gives the usual result."""
    import ctypes
    hip = ctypes.CDLL("libamdhip64.so.7")
    w = workload("c1_small_fp64")
    base = run_gpu(w, "fp32")
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    m = B.Matcher(w["params"], "fp32")
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    torch.cuda.synchronize()
    assert hip.hipSetDevice(ctypes.c_int(1 << 20)) != 0
    with pytest.raises(B.TrdError) as e:
        m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    assert e.value.code == B.TRD_EDEVICE
    out = pu.to_numpy(m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"]))
    torch.cuda.synchronize()
    m.close()
    for k in ("idx", "p", "cov", "status"):
        assert np.array_equal(out[k], base[k], equal_nan=True), k
