"""Pins of the oracle's residual maps (Sect. 2, steps 4 and 5: residuals of
the distorted TPC clusters against reference tracks, collected per
sub-volume, and one distortion vector per sub-volume).

- no distortion, exact clusters, the true track as reference: every residual
  and every voxel's vector is zero, and every cluster is counted;
- a smooth distortion, exact clusters, the true track: each voxel's vector
  equals the least-squares solution built here in numpy from the generator's
  own field values and track angles (second-order terms only);
- with cluster noise and the true track as reference: all three components
  scatter around the voxel means of the field within their statistical
  error, without bias;
- with the TRD-only refit as reference the maps are only as good as its
  extrapolation 200 cm inwards (the paper interpolates between inner and
  outer refits): checked for the zero-distortion case, where the voxel means
  of the residuals must vanish within their errors.
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import synth

NX, NY, NZ = O.VOXELS


def truth_reference(w):
    T = w["truth"]
    p = np.stack([T["y"][0], T["z"][0], T["snp"][0], T["tgl"][0], T["qpt"][0]])
    ok = np.isfinite(p).all(axis=0)
    return dict(p=np.where(ok, p, 0.0), x=np.where(ok, T["x"][0], 290.0),
                sector=np.where(ok, T["sec"][0], 0).astype(np.int32), status=np.where(ok, 0, 1).astype(np.uint32))


def voxel_ids(cl, xr):
    tan10 = math.tan(math.pi / 18)
    t = cl["tpc"]
    ix = np.clip(np.floor((xr - t["x_in"]) / (t["x_out"] - t["x_in"]) * NX), 0, NX - 1).astype(int)
    iy = np.clip(np.floor((cl["y_true"] / xr / tan10 + 1) * 0.5 * NY), 0, NY - 1).astype(int)
    iz = np.clip(np.floor((cl["z_true"] / xr + 1) * 0.5 * NZ), 0, NZ - 1).astype(int)
    return ((cl["sector"] * NX + ix) * NY + iy) * NZ + iz


def linear_model_solution(cl):
    """Per voxel (dY, dZ, dX): least squares of r_y = dY - t_y dX,
    r_z = dZ - t_z dX over the generator's field values and track angles."""
    v = voxel_ids(cl, cl["x_rows"][cl["row"]])
    ty, tz = cl["ty_true"], cl["tz_true"]
    ry = cl["dY"] - ty * cl["dX"]
    rz = cl["dZ"] - tz * cl["dX"]
    ref = np.full((18 * NX * NY * NZ, 3), np.nan)
    for k in np.unique(v):
        sel = v == k
        m = int(sel.sum())
        if m < O.VOXEL_MIN:
            continue
        A = np.zeros((2 * m, 3))
        A[:m, 0], A[:m, 2] = 1.0, -ty[sel]
        A[m:, 1], A[m:, 2] = 1.0, -tz[sel]
        ref[k] = np.linalg.lstsq(A, np.concatenate([ry[sel], rz[sel]]), rcond=None)[0]
    return ref


def exact_frame(n, seed, field):
    P = synth.default_params()
    g = synth.generate_group(np.random.default_rng(seed), P, n, fake_ratio=0.0, noise_free=True, ms=False)
    w = synth._concat_groups([g], P)
    return P, w, synth.tpc_clusters(w, seed, field=field, noise_free=True)


def test_no_distortion_gives_zero_everywhere():
    P, w, cl = exact_frame(20000, 3, False)
    s = O.residual_sums(P, truth_reference(w), cl)
    d = O.voxel_solve(s, cl["tpc"])
    assert s[:, 0].sum() == cl["n_clusters"]
    assert np.abs(s[:, 4:]).max() < 1e-8
    ok = np.isfinite(d[:, 0])
    assert ok.sum() == 18 * NX * NY * NZ
    assert np.abs(d[ok, :3]).max() < 1e-9


def test_smooth_distortion_matches_the_linear_model():
    P, w, cl = exact_frame(20000, 5, True)
    s = O.residual_sums(P, truth_reference(w), cl)
    d = O.voxel_solve(s, cl["tpc"])
    # the same least squares from the generator's field values and angles
    ref = linear_model_solution(cl)
    nv = 18 * NX * NY * NZ
    got = d[:, [1, 2, 0]]
    ok = np.isfinite(ref[:, 0]) & np.isfinite(got[:, 0])
    assert ok.sum() > 0.95 * nv
    err = np.abs(got[ok] - ref[ok]).max(axis=0)
    # second-order terms: dX^2 / (2R) and the field's change over dX
    assert np.all(err < np.array([5e-3, 5e-3, 2e-2])), err


def test_noisy_clusters_true_reference():
    P = synth.default_params()
    g = synth.generate_group(np.random.default_rng(9), P, 20000, fake_ratio=0.0, ms=False)
    w = synth._concat_groups([g], P)
    cl = synth.tpc_clusters(w, 9)
    s = O.residual_sums(P, truth_reference(w), cl)
    d = O.voxel_solve(s, cl["tpc"])
    ref = linear_model_solution(cl)
    got = d[:, [1, 2, 0]]
    ok = np.isfinite(ref[:, 0]) & np.isfinite(got[:, 0]) & (s[:, 0] >= 200)
    assert ok.sum() > 0.8 * ref.shape[0]
    diff = got[ok] - ref[ok]
    # cluster noise 0.05 cm over a few hundred clusters; dX through the
    # spread of the track angles in the voxel
    assert np.all(np.abs(np.median(diff, axis=0)) < np.array([0.005, 0.005, 0.05])), np.median(diff, axis=0)
    assert np.all(np.percentile(np.abs(diff), 90, axis=0) < np.array([0.05, 0.05, 0.5])), \
        np.percentile(np.abs(diff), 90, axis=0)


def test_refit_reference_without_distortion():
    P = synth.default_params()
    g = synth.generate_group(np.random.default_rng(10), P, 20000, fake_ratio=0.0)
    w = synth._concat_groups([g], P)
    cl = synth.tpc_clusters(w, 10, field=False)
    m = O.match(P, w, threads=0)
    r = O.refit(P, m, m["idx"], w)
    s = O.residual_sums(P, r, cl)
    ok = s[:, 0] >= 200
    # mean residuals per voxel against their own scatter
    mu = s[ok, 4:6] / s[ok, 0:1]
    var = s[ok, 7:8] / s[ok, 0:1] / 2.0
    z = mu / np.sqrt(var / s[ok, 0:1])
    assert abs(np.median(z)) < 0.5, np.median(z)
