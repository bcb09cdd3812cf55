"""Residual maps (Sect. 2, steps 4-5) on the HIP path against the oracle's
maps, through the C ABI, on the same reference tracks and clusters."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def device_clusters(cl):
    dev = torch.device("cuda", 0)
    rs = (cl["sector"].astype(np.int64) << 16) | cl["row"].astype(np.int64)
    return dict(y=torch.from_numpy(cl["y"].astype(np.float32)).to(dev),
                z=torch.from_numpy(cl["z"].astype(np.float32)).to(dev),
                row_sec=torch.from_numpy(rs.astype(np.int32)).to(dev),
                first=torch.from_numpy(cl["first"].astype(np.int64)).to(dev))


def gpu_chain(w, cl, prec):
    """match -> TRD-only refit -> residual sums and vectors, all on the GPU."""
    d = B.device_inputs(synth.to_device_layout(w), prec)
    m = B.Matcher(w["params"], prec)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    mo = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    r = m.refit(mo, d["y"], d["z"], d["det_row"])
    sums, dist = m.residual_map(r, device_clusters(cl))
    torch.cuda.synchronize()
    ref = {k: r[k].cpu().numpy() for k in ("p", "x", "sector", "status")}
    out = (sums.cpu().numpy(), dist.cpu().numpy(), ref, m, d, r)
    return out


def compare_maps(s_gpu, d_gpu, s_ref, n_cl, prec):
    """Every voxel with a solution.  Double: identical counts, sums within
    1e-10 relative (they add the same terms in another order), the solutions
    of both sets of sums within 1e-10 cm, and the kernel's own float solution
    within float rounding of that.  Float: voxel membership can differ at bin
    edges between the float and the double track, so the counts agree to a
    handful of clusters and the vectors to the float track's error carried
    through the fit."""
    d_ref = O.voxel_solve(s_ref, B.TPC_ROWS | {"n_rows": 64})
    if prec == "fp64":
        assert np.array_equal(s_gpu[:, 0], s_ref[:, 0])
        # sums of up to ~1e4 terms of either sign, added in another order
        assert np.all(np.abs(s_gpu - s_ref) <= 1e-10 * np.maximum(np.abs(s_ref), 1.0)), \
            np.abs(s_gpu - s_ref).max()
        d_mine = O.voxel_solve(s_gpu, B.TPC_ROWS | {"n_rows": 64})
        ok = np.isfinite(d_ref[:, 0])
        assert np.array_equal(ok, np.isfinite(d_mine[:, 0])) and ok.sum() > 0.5 * len(ok)
        err = np.abs(d_mine[ok, :3] - d_ref[ok, :3])
        assert err.max() <= 1e-10, err.max(axis=0)
        # the kernel's float4 output: its own double solve rounded to float
        f_err = np.abs(d_gpu[ok, :3].astype(np.float64) - d_ref[ok, :3])
        assert np.all(f_err <= 1e-6 * np.maximum(np.abs(d_ref[ok, :3]), 1.0)), f_err.max(axis=0)
        return err.max(axis=0)
    # voxel membership is a discrete decision on the track point: a cluster
    # whose point lies at a voxel edge within the float track's error may
    # fall on the other side; such moves are counted, and every voxel that
    # kept exactly its clusters' count is held to the float arithmetic
    moved = np.abs(s_gpu[:, 0] - s_ref[:, 0]).sum() / 2
    assert moved <= max(3, 1e-4 * n_cl), moved
    ok = np.isfinite(d_ref[:, 0]) & np.isfinite(d_gpu[:, 0]) & (s_ref[:, 0] >= 200)
    assert ok.sum() > 0.5 * len(ok)
    same = ok & (s_gpu[:, 0] == s_ref[:, 0])
    err = np.abs(d_gpu[ok, :3].astype(np.float64) - d_ref[ok, :3])
    err_same = np.abs(d_gpu[same, :3].astype(np.float64) - d_ref[same, :3])
    print(f"float map: {moved:.0f} clusters moved, {ok.sum() - same.sum()} of {ok.sum()} voxels changed count;"
          f" error max over unchanged voxels {err_same.max(axis=0)}, 99th percentile over all"
          f" {np.percentile(err, 99, axis=0)}")
    assert same.sum() > 0.5 * ok.sum()
    assert np.all(err_same.max(axis=0) < np.array([5e-2, 5e-3, 5e-3])), err_same.max(axis=0)
    assert np.all(np.percentile(err, 99, axis=0) < np.array([5e-2, 5e-3, 5e-3])), np.percentile(err, 99, axis=0)
    return err_same.max(axis=0)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_residual_map_frame(prec):
    w = synth.generate("c2_frame_20k")
    cl = synth.tpc_clusters(w, 4)
    s_gpu, d_gpu, ref, m, _, _ = gpu_chain(w, cl, prec)
    m.close()
    s_ref = O.residual_sums(w["params"], ref, cl)
    print(compare_maps(s_gpu, d_gpu, s_ref, cl["n_clusters"], prec))


def test_batches_accumulate():
    w = synth.generate("c2_frame_20k")
    cl = synth.tpc_clusters(w, 4)
    s_all, _, ref, m, d, r = gpu_chain(w, cl, "fp32")
    dc = device_clusters(cl)
    half = w["n_tracks"] // 2
    first = dc["first"]
    parts = None
    for lo, hi in ((0, half), (half, w["n_tracks"])):
        sub_ref = {k: (r[k][:, lo:hi].contiguous() if r[k].dim() == 2 else r[k][lo:hi].contiguous())
                   for k in ("p", "x", "sector", "status")}
        sub_cl = dict(dc, first=first[lo:hi + 1].contiguous())
        parts, _ = m.residual_map(sub_ref, sub_cl, sums=parts)
    torch.cuda.synchronize()
    m.close()
    p = parts.cpu().numpy()
    assert np.array_equal(p[:, 0], s_all[:, 0])
    assert np.allclose(p, s_all, rtol=1e-5, atol=1e-3)


def test_no_distortion_exact_clusters_true_reference():
    P = synth.default_params()
    g = synth.generate_group(np.random.default_rng(3), P, 5000, fake_ratio=0.0, noise_free=True, ms=False)
    w = synth._concat_groups([g], P)
    cl = synth.tpc_clusters(w, 3, field=False, noise_free=True)
    T = w["truth"]
    p = np.stack([T["y"][0], T["z"][0], T["snp"][0], T["tgl"][0], T["qpt"][0]])
    good = np.isfinite(p).all(axis=0)
    dev = torch.device("cuda", 0)
    ref = dict(p=torch.from_numpy(np.where(good, p, 0.0).astype(np.float32)).to(dev),
               x=torch.from_numpy(np.where(good, 290.0, 290.0).astype(np.float32)).to(dev),
               sector=torch.from_numpy(np.where(good, T["sec"][0], 0).astype(np.int32)).to(dev),
               status=torch.from_numpy(np.where(good, 0, 1).astype(np.int32)).to(dev))
    m = B.Matcher(P, "fp32")
    sums, dist = m.residual_map(ref, device_clusters(cl))
    torch.cuda.synchronize()
    m.close()
    s = sums.cpu().numpy()
    assert s[:, 0].sum() == cl["n_clusters"]
    # float track and float clusters: residuals of a few 1e-5 cm at most
    assert np.abs(s[:, 4:6] / np.maximum(s[:, :1], 1)).max() < 1e-4


def test_residual_map_distortion_batch():
    """The 450k batch matched and refitted in full; the map of the clusters of
    its first 100k tracks (the oracle's sums on the GPU's reference tracks)."""
    w = synth.generate("c5_distortion_450k")
    sub = np.arange(100000)
    cl = synth.tpc_clusters(w, 6, tracks=sub)
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    m = B.Matcher(w["params"], "fp32")
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    mo = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    r = m.refit(mo, d["y"], d["z"], d["det_row"])
    rs = {k: (r[k][:, :sub.size].contiguous() if r[k].dim() == 2 else r[k][:sub.size].contiguous())
          for k in ("p", "x", "sector", "status")}
    sums, dist = m.residual_map(rs, device_clusters(cl))
    torch.cuda.synchronize()
    m.close()
    ref = {k: v.cpu().numpy() for k, v in rs.items()}
    s_ref = O.residual_sums(w["params"], ref, cl)
    print(compare_maps(sums.cpu().numpy(), dist.cpu().numpy(), s_ref, cl["n_clusters"], "fp32"))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_chain_end_to_end_against_the_oracle_chain(prec):
    """GPU match -> GPU refit -> GPU map against oracle match -> oracle refit
    -> oracle map of the same frame, with no GPU output fed to the oracle.
    Tracks whose matching carries a decision-margin flag are left out of both
    maps (their tracklets may legitimately differ)."""
    w = synth.generate("c2_frame_20k")
    cl = synth.tpc_clusters(w, 4)
    P = w["params"]
    om = O.match(P, w, threads=0, margins=pu.MARGINS[prec])
    flagged = om["flags"] != 0
    orf = O.refit(P, om, om["idx"], w)
    orf = dict(orf, status=np.where(flagged, orf["status"] | 1, orf["status"]).astype(np.uint32))
    s_ref = O.residual_sums(P, orf, cl)
    d = B.device_inputs(synth.to_device_layout(w), prec)
    m = B.Matcher(P, prec)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    mo = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    r = m.refit(mo, d["y"], d["z"], d["det_row"])
    excl = torch.from_numpy(flagged.astype(np.int32)).to(r["status"].device)
    r["status"] = (r["status"].to(torch.int32) | excl).to(r["status"].dtype)
    sums, dist = m.residual_map(r, device_clusters(cl))
    torch.cuda.synchronize()
    gidx = mo["idx"].cpu().numpy()
    m.close()
    assert np.array_equal(gidx[:, ~flagged], om["idx"][:, ~flagged])
    print(compare_maps(sums.cpu().numpy(), dist.cpu().numpy(), s_ref, cl["n_clusters"], prec))
