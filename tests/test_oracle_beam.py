"""Pins of the oracle's multi-hypothesis matching (Sect. 3, Fig. 2: the best
N_candidates hypotheses of a layer seed the next one).

- one hypothesis with the no-tracklet cost at the chi2 cut is the single
  best-candidate matcher, bit for bit;
- with more hypotheses kept than there are paths, the answer is the cheapest
  of all paths, found here by enumerating every path in Python from the
  oracle's single steps (propagation, rotation, scattering, update);
- binned and brute-force candidate sets give the same answer;
- a zero no-tracklet cost makes the empty path the cheapest.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import synth

KEYS = ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status")


def _beam(P, n_hyp, penalty=None):
    Q = dict(P)
    Q["n_hyp"] = n_hyp
    Q["chi2_penalty"] = P["chi2_max"] if penalty is None else penalty
    return Q


@pytest.mark.parametrize("name,over", [
    ("c1_small_fp64", {}),
    ("c1_small_fp64", dict(tilt_on=True)),
    ("c2_frame_20k", {}),
])
def test_one_hypothesis_is_the_single_best_matcher(name, over):
    w = synth.generate(name)
    P = dict(w["params"])
    if over.get("tilt_on"):
        P["tilt"] = [synth.tilt_pm2deg()[l] for l in range(6)]
        rng = np.random.default_rng(5)
        P["dx_chamber"] = rng.uniform(-0.5, 0.5, 540)
    sl = np.arange(min(w["n_tracks"], 4000))
    a = O.match(P, w, threads=0, track_slice=sl)
    b = O.match(_beam(P, 1), w, threads=0, track_slice=sl)
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k
    assert (a["n_match"] > 0).mean() > 0.5


def test_binned_equals_brute_force_with_three_hypotheses():
    w = synth.generate("c1_small_fp64")
    P = _beam(w["params"], 3)
    a = O.match(P, w, threads=0)
    b = O.match(P, w, mode="brute", threads=0)
    for k in KEYS:
        assert np.array_equal(a[k], b[k], equal_nan=True), k


def test_zero_penalty_prefers_no_tracklets():
    w = synth.generate("c1_small_fp64")
    r = O.match(_beam(w["params"], 4, penalty=0.0), w, threads=0)
    assert np.all(r["n_match"] == 0) and np.all(r["idx"] == -1)


# ---- exhaustive enumeration on tiny inputs -----------------------------------

def _road(P, p, C, l):
    """Road quantities of a predicted state (the single-matcher definition)."""
    s, t = p[2], p[3]
    f = math.sqrt(1.0 - s * s)
    tau = P["tilt"][l]
    sy = P["sigma_y"][0] + P["sigma_y"][1] * s + P["sigma_y"][2] * s * s
    vz = P["pad_len"] ** 2 / 12.0
    Syy = C[0, 0] + 2 * tau * C[0, 1] + tau * tau * C[1, 1] + sy * sy
    Syz = C[0, 1] + tau * C[1, 1]
    Szz = C[1, 1] + vz
    sdy = P["sigma_dy"][0] + P["sigma_dy"][1] * s + P["sigma_dy"][2] * s * s
    gdy = P["n_sigma_dy"] * math.sqrt(sdy * sdy + P["drift_len"] ** 2 * C[2, 2] / f ** 6)
    S = np.array([[Syy, Syz], [Syz, Szz]])
    return dict(tau=tau, S=S, Ry=P["n_sigma_road"] * math.sqrt(Syy), Rz=P["n_sigma_road"] * math.sqrt(Szz),
                dytrk=P["drift_len"] * (s / f - P["tan_psi"]), gdy=gdy, vy=sy * sy, vz=vz)


def _predict(P, p, C, x, sec, l):
    ok, p, c, x, _ = O.propagate(P, p, O.pack(C), x, P["x_layer"][l])
    if not ok:
        return None
    for nrot in range(3):
        if abs(p[0]) <= P["x_layer"][l] * math.tan(math.pi / 18):
            break
        if nrot == 2:
            return None
        up = p[0] > 0
        ok, p, c, x, _ = O.rotate(P, p, c, x, (1 if up else -1) * 2 * math.pi / 18)
        if not ok:
            return None
        sec = (sec + (1 if up else 17)) % 18
        ok, p, c, x, _ = O.propagate(P, p, c, x, P["x_layer"][l])
        if not ok:
            return None
    c = O.add_ms(P, p, c)
    return p, O.unpack(c), x, sec


def _all_paths(P, w, i):
    """Every path of track i: (cost, idx tuple, final p, final packed cov)."""
    out = []
    pen = P["chi2_penalty"]

    def rec(l, p, C, x, sec, live, cost, path):
        if l == 6:
            out.append((cost, tuple(path), p, O.pack(C)))
            return
        if live:
            pr = _predict(P, p, C, x, sec, l)
            if pr is None:
                live = False
            else:
                p, C, x, sec = pr
        kids = []
        if live:
            r = _road(P, p, C, l)
            Si = np.linalg.inv(r["S"])
            det = sec * 30 + l
            for j in range(w["n_tracklets"]):
                dj = int(w["tkl_det_row"][j]) >> 5
                if dj - (dj // 30) * 30 - ((dj % 30) // 6) * 6 != l or dj // 30 != sec:
                    continue
                yj, zj, dyj = w["tkl_y"][j], w["tkl_z"][j], w["tkl_dy"][j]
                ry = yj - (p[0] + r["tau"] * (p[1] - zj))
                rz = zj - p[1]
                res = np.array([ry, rz])
                c2 = float(res @ Si @ res)
                if (abs(ry) <= r["Ry"] and abs(rz) <= r["Rz"] and abs(dyj - r["dytrk"]) <= r["gdy"]
                        and c2 <= P["chi2_max"]):
                    kids.append((j, c2, ry, rz, r))
        for j, c2, ry, rz, r in kids:
            p2, c2v = O.update(p, O.pack(C), ry, rz, r["tau"], r["vy"], r["vz"])
            C2 = O.unpack(c2v)
            ok = abs(p2[2]) < P["snp_max"]
            rec(l + 1, p2, C2, x, sec, ok, cost + c2, path + [j])
        rec(l + 1, p, C, x, sec, live, cost + pen, path + [-1])

    p0 = w["p"][:, i].copy()
    rec(0, p0, O.unpack(w["cov"][:, i]), float(w["x"][i]), int(w["sector"][i]), True, 0.0, [])
    return out


def _tiny(seed):
    """One track; its own tracklets in layers 0, 1 and 3, plus a second
    tracklet near the first one in layer 0."""
    P = synth.default_params()
    rng = np.random.default_rng(seed)
    g = synth.generate_group(rng, P, 1, fake_ratio=0.0, ineff_frac=0.0)
    w = synth._concat_groups([g], P)
    keep = [int(w["true_idx"][l, 0]) for l in (0, 1, 3) if w["true_idx"][l, 0] >= 0]
    j0 = int(w["true_idx"][0, 0])
    sel = np.array(keep + ([j0] if j0 >= 0 else []))
    for k in ("tkl_y", "tkl_z", "tkl_dy", "tkl_det_row", "tkl_group"):
        w[k] = np.ascontiguousarray(w[k][sel])
    if j0 >= 0:
        w["tkl_y"] = w["tkl_y"].copy()
        w["tkl_y"][-1] += rng.uniform(0.05, 0.3) * (1 if rng.random() < 0.5 else -1)
        w["tkl_dy"] = w["tkl_dy"].copy()
        w["tkl_dy"][-1] += rng.normal(0, 0.02)
    w["n_tracklets"] = int(sel.size)
    return P, w


@pytest.mark.parametrize("penalty", [13.8155, 4.0])
def test_more_hypotheses_than_paths_finds_the_cheapest_path(penalty):
    checked = 0
    for seed in range(40):
        P, w = _tiny(seed)
        P = _beam(P, 16, penalty)
        paths = _all_paths(P, w, 0)
        assert len(paths) <= 16
        if len(paths) < 4:
            continue
        costs = sorted(c for c, *_ in paths)
        if costs[1] - costs[0] < 1e-9:
            continue
        best = min(paths, key=lambda t: t[0])
        r = O.match(P, w, threads=0)
        assert tuple(r["idx"][:, 0]) == best[1], (seed, best, r["idx"][:, 0])
        np.testing.assert_allclose(r["p"][:, 0], best[2], rtol=1e-12, atol=1e-12)
        np.testing.assert_allclose(r["cov"][:, 0], best[3], rtol=1e-10, atol=1e-15)
        nm = int(sum(j >= 0 for j in best[1]))
        assert r["n_match"][0] == nm
        assert r["chi2"][0] + penalty * (6 - nm) == pytest.approx(best[0], rel=1e-12)
        checked += 1
    assert checked >= 10
