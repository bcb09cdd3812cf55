#!/usr/bin/env python3
"""Throughput of the TRD matching hot path on one MI355X.

One step = bin all tracklets of the batch (keys + histogram, scan, stable
scatter) and match every seed track through the six layers, with the inputs
already resident in device memory.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "k_match_c5_distortion_450k_fp32.md")
SOURCES = ("trd_api.hip", "trd_bin.hip", "trd_match.hip", "trd_internal.h")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def match_alg_bytes(n_trk, n_tkl, n_cells, prec):
    """Algorithmic bytes of one match launch: track state in and out, each
    binned tracklet record once, the cell offsets once."""
    f = 8 if prec == "fp64" else 4
    trk_in = 21 * f + 4 + 4                 # p, cov, x; sector, group
    trk_out = 21 * f + f + 6 * 4 + 3 * 4    # p, cov, x; chi2; idx; sector, n_match, status
    return n_trk * (trk_in + trk_out) + n_tkl * 16 + (n_cells + 1) * 4


def bin_alg_bytes(n_tkl, n_cells):
    """Algorithmic bytes of the binning: read y, z, dy, det_row, group (20 B)
    twice (histogram, scatter), write the 16 B record, count/offset traffic."""
    return n_tkl * (20 + 20 + 16) + n_cells * 16


def source_hash():
    """sha256 of the HIP sources the library is built from."""
    h = hashlib.sha256()
    for f in SOURCES:
        with open(os.path.join(ROOT, "paper_2003_03174_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _profiled(key):
    """A per-launch figure of k_match from the committed counter summary, if
    it was taken on the current sources (else None)."""
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    m = re.search(key + r":\s*([0-9.eE+]+)", text)
    s = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    if not m or not s or s.group(1) != source_hash():
        return None
    return float(m.group(1))


def profiled_traffic():
    """HBM bytes per launch of k_match (FETCH_SIZE and WRITE_SIZE, scaled)."""
    return _profiled("traffic_bytes_per_launch")


def profiled_valu():
    """Share of the VALU issue slots k_match used and its active-lane share."""
    a, b = _profiled("valu_issue_frac"), _profiled("valu_lane_frac")
    if a is None or b is None:
        return None
    return {"issue_frac": a, "lane_frac": b, "source": os.path.relpath(PROFILE, ROOT)}


def run_gpu(w, prec, steps, warmup, block_size=0, search_lanes=0, graph=False, d=None, flags=0, fused=True):
    import torch
    from paper_2003_03174_amd import binding as B
    from paper_2003_03174_amd import synth

    if d is None:
        d = B.device_inputs(synth.to_device_layout(w), prec)
    n = w["n_tracks"]
    if not graph:
        flags |= B.TRD_CFG_TIME_KERNEL
    m = B.Matcher(w["params"], prec, block_size=block_size, search_lanes=search_lanes, flags=flags)
    m.reserve(w["n_tracklets"], w["n_groups"], n)
    out = m.alloc_results(n, chi2_layer=False)
    stream = torch.cuda.current_stream()

    def load_and_match():
        m.load_and_match(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"], d["p"], d["cov"],
                         d["x"], d["sector"], tgroup=d["group"], out=out)

    def body():
        if fused:
            load_and_match()
        else:
            m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
            m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)

    g = None
    if graph:
        # bin + match of the whole batch captured once, replayed per step
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

    def step(evs=None):
        if evs:
            evs[0].record(stream)
        if g is not None:
            g.replay()
            if evs:
                evs[1].record(stream)
        elif fused:
            load_and_match()
            if evs:
                evs[1].record(stream)
        else:
            m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
            if evs:
                evs[1].record(stream)
            m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)
        if evs:
            evs[2].record(stream)

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    if not graph:
        m.kernel_times()   # drop the warm-up launches
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ktimes = m.kernel_times() if not graph else []
    # per-step latency from events around each step, in a pass of its own
    # after the timed steps: an event recorded between steps is a packet of
    # its own on the stream, which the timed steps do without
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(steps)]
    for k in range(steps):
        step(evs[k])
    torch.cuda.synchronize()
    if not graph:
        m.kernel_times()
    t_bin = [e[0].elapsed_time(e[1]) for e in evs]
    t_match = [e[1].elapsed_time(e[2]) for e in evs]
    t_step = [e[0].elapsed_time(e[2]) for e in evs]
    if fused and not graph:
        # the fused call has no boundary between binning and matching: the
        # split comes from separate calls after the timed steps
        sp = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(min(steps, 10))]
        for e in sp:
            e[0].record(stream)
            m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
            e[1].record(stream)
            m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)
            e[2].record(stream)
        torch.cuda.synchronize()
        m.kernel_times()
        t_bin = [e[0].elapsed_time(e[1]) for e in sp]
        t_match = [e[1].elapsed_time(e[2]) for e in sp]
    if graph:
        # a replayed graph has no event between its kernels: the match
        # kernel's own duration comes from a matcher with the same launch
        # shape that records it, stepping eagerly after the timed replays,
        # and the step is not split into binning and matching
        t_bin = t_match = None
        mk = B.Matcher(w["params"], prec, block_size=block_size, search_lanes=search_lanes,
                       flags=flags | B.TRD_CFG_TIME_KERNEL)
        mk.reserve(w["n_tracklets"], w["n_groups"], n)
        outk = mk.alloc_results(n, chi2_layer=False)
        for k in range(warmup + steps):
            if k == warmup:
                torch.cuda.synchronize()
                mk.kernel_times()
            mk.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
            mk.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=outk)
        torch.cuda.synchronize()
        ktimes = mk.kernel_times()
        mk.close()
    st = out["status"].cpu().numpy()
    nm = out["n_match"].cpu().numpy()
    # TRD-only refit of the last step's matches (not part of the step)
    ref_ms = []
    full = m.alloc_results(n)
    m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=full)
    for k in range(4):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.refit(full, d["y"], d["z"], d["det_row"])
        e1.record(stream)
        torch.cuda.synchronize()
        if k:
            ref_ms.append(e0.elapsed_time(e1))
    last = {k: (v.cpu().numpy() if v is not None else None) for k, v in full.items()}
    res = dict(wall_ms_per_step=1e3 * wall / steps, bin_ms=t_bin, match_ms=t_match, step_ms=t_step,
               refit_ms=ref_ms, result=last,
               kernel_ms=ktimes,
               n_fallback=int(((st & B.TRK_FP64_FALLBACK) != 0).sum()),
               n_ge2=int((nm >= 2).sum()))
    m.close()
    return res


def pct(v, q):
    v = sorted(v)
    k = min(len(v) - 1, max(0, int(math.ceil(q / 100.0 * len(v))) - 1))
    return v[k]


def cpu_model():
    """The host CPU's model name and its logical core count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, os.cpu_count()


def cpu_baseline(w, gpu=None, prec="fp32", budget_s=6.0, runs=3):
    """The FP64 oracle on the host cores: binning of all tracklets plus the
    matching of a bounded sample of tracks, extrapolated to the batch (median
    of `runs` runs).  With `gpu` (the device results of the whole batch) the
    oracle's tracks of a 3,000-track sample also give the error of the device
    path per quantity and the decision-margin flag counts."""
    import numpy as np
    from oracle import oracle as O

    P = w["params"]
    n = w["n_tracks"]
    cores = int(O.lib().oracle_max_threads())
    t0 = time.perf_counter()
    O.bin_tracklets(P, w)
    t_bin = time.perf_counter() - t0
    probe = np.arange(0, n, max(1, n // 2000))
    t0 = time.perf_counter()
    O.match(P, w, threads=cores, track_slice=probe)
    t_probe = max(time.perf_counter() - t0 - t_bin, 1e-6) / probe.size
    ns = int(min(n, max(probe.size, budget_s / t_probe)))
    sample = np.arange(0, n, max(1, n // ns))[:ns]
    ests, calls = [], []
    for _ in range(runs):
        t0 = time.perf_counter()
        O.match(P, w, threads=cores, track_slice=sample)
        t_call = time.perf_counter() - t0
        calls.append(t_call)
        ests.append(t_bin + max(t_call - t_bin, 1e-9) / sample.size * n)
    est = float(np.median(ests))
    # one thread: the binning and a smaller sample, same extrapolation
    s1 = np.arange(0, n, max(1, n // 20000))
    t0 = time.perf_counter()
    O.match(P, w, threads=1, track_slice=s1)
    t_one = time.perf_counter() - t0
    t0 = time.perf_counter()
    O.bin_tracklets(P, w)
    t_bin1 = time.perf_counter() - t0   # the binning is single-threaded in the oracle
    est1 = t_bin1 + max(t_one - t_bin1, 1e-9) / s1.size * n
    model, logical = cpu_model()
    out = dict(value=n / est, unit="tracks/s", cores=cores, kind="oracle",
               cpu_model=model, logical_cpus=logical,
               runs=[n / e for e in ests],
               value_1_thread=n / est1,
               sample=(f"binning of all {w['n_tracklets']} tracklets ({t_bin:.2f} s) + matching of "
                       f"{sample.size} of {n} tracks (every {max(1, n // ns)}th, median of {runs} runs, "
                       f"{float(np.median(calls)) - t_bin:.2f} s), extrapolated to the whole batch; "
                       f"1 thread: {s1.size} tracks"))
    if gpu is not None:
        out["parity"] = parity_sample(O, w, gpu, prec, cores)
    return out


def parity_sample(O, w, gpu, prec, cores, n_sample=3000):
    """Error of the device results against the FP64 oracle on sampled tracks,
    per quantity (relative, floors 10 cm, 10 cm, 0.1, 0.1, 0.1 c/GeV), and the
    oracle's decision-margin flags (the exempt tracks)."""
    import numpy as np
    from tests import parity_util as pu

    sel = np.sort(np.random.default_rng(0).choice(w["n_tracks"], min(n_sample, w["n_tracks"]),
                                                  replace=False))
    hyp = int(w["params"].get("n_hyp", 0)) > 0
    margins = (pu.BEAM_MARGINS if hyp else pu.MARGINS)[prec]
    ref = O.match(w["params"], w, threads=cores, margins=margins, track_slice=sel)
    rep = pu.compare(ref, gpu, prec, sel=sel, max_flag_share=pu.MAX_FLAG_SHARE_BEAM_WIDE if hyp else None)
    names = ("y", "z", "sin_phi", "tan_lambda", "q_over_pt")
    return {
        "n_sampled": int(sel.size),
        "tolerance": {"state": pu.STATE_TOL[prec], "cov": pu.COV_TOL[prec], "chi2": pu.chi2_tol(prec)},
        "max_rel_err": dict(zip(names, rep.state_err_by_comp)),
        "max_rel_err_x": rep.x_err,
        "max_cov_err": rep.cov_err,
        "max_chi2_err": rep.chi2_err,
        "idx_mismatch": rep.idx_mismatch + rep.idx_mismatch_flagged_prefix,
        "status_mismatch": rep.status_mismatch,
        "flagged": dict(rep.flag_counts, total=rep.n_flagged, near_chi2_cut_only=rep.n_flag_cut_only),
        "ok": bool(rep.ok),
    }


def residual_bench(args):
    """Residual maps of the 450k batch (one map's worth of tracks): match and
    refit on the GPU, clusters on 64 pad rows per track, then the voxel sums
    and the per-voxel fit, timed with HIP events."""
    import numpy as np
    import torch
    from paper_2003_03174_amd import binding as B
    from paper_2003_03174_amd import synth

    log("generating c5_distortion_450k and its TPC clusters")
    w = synth.load_workload("c5_distortion_450k")
    cl = synth.tpc_clusters(w, 6)
    n, m_cl = w["n_tracks"], cl["n_clusters"]
    dev = torch.device("cuda", 0)
    rs = (cl["sector"].astype(np.int64) << 16) | cl["row"].astype(np.int64)
    dc = dict(y=torch.from_numpy(cl["y"].astype(np.float32)).to(dev),
              z=torch.from_numpy(cl["z"].astype(np.float32)).to(dev),
              row_sec=torch.from_numpy(rs.astype(np.int32)).to(dev),
              first=torch.from_numpy(cl["first"]).to(dev))
    d = B.device_inputs(synth.to_device_layout(w), "fp32")
    m = B.Matcher(w["params"], "fp32")
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    mo = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    r = m.refit(mo, d["y"], d["z"], d["det_row"])
    nx, ny, nz = B.VOXELS
    sums = torch.zeros((18 * nx * ny * nz, 8), dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    ts = []
    for k in range(args.warmup + args.steps):
        sums.zero_()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, dist = m.residual_map(r, dc, sums=sums)
        e1.record(stream)
        torch.cuda.synchronize()
        if k >= args.warmup:
            ts.append(e0.elapsed_time(e1))
    ms = sum(ts) / len(ts)
    dd = dist.cpu().numpy()
    m.close()
    # algorithmic bytes: clusters (y, z, row/sector: 12 B) + references (28 B) + sums
    ab = m_cl * 12 + n * 28 + sums.numel() * 8 * 2
    line = {"metric": "TPC clusters accumulated into residual maps per second", "value": m_cl / (ms * 1e-3),
            "unit": "clusters/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": f"c5_distortion_450k refitted tracks, {m_cl} clusters on 64 pad rows, "
                                   f"{18 * nx * ny * nz} voxels", "step": "residual sums + voxel fit"},
            "voxels_solved": int(np.isfinite(dd[:, 0]).sum()),
            "roofline": {"bound": "hbm", "achieved": ab / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": ab / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                         "kernel": "k_residual_sums + k_voxel_solve", "alg_bytes_per_launch": ab}}
    print(json.dumps(line), flush=True)


def serve_bench(args):
    """Poisson stream of frames served by continuous batching (float path,
    two slots) against static batching with the plain double kernel."""
    import numpy as np
    import torch
    from paper_2003_03174_amd import serve, synth

    P = synth.default_params()
    rng = np.random.default_rng(3)
    n_pool = args.serve_pool
    sizes = np.maximum(1, np.round(rng.lognormal(math.log(15000), 0.6, n_pool))).astype(int)
    ss = np.random.SeedSequence(3).spawn(n_pool)
    log(f"generating {n_pool} frames (lognormal tracks, median 15000)")

    def make_pool(sizes, ss):
        out = []
        for n, s in zip(sizes, ss):
            g = synth.generate_group(np.random.default_rng(s), P, int(n), fake_ratio=0.5, ineff_frac=0.1)
            w = synth._concat_groups([g], P)
            out.append((w["n_tracks"], w["n_tracklets"], serve.frame_arrays(w, pinned=True)))
        return out

    pool = make_pool(sizes, ss)
    # the warm-up stream: other frames of the same size mix, one second at
    # the served rate, so that every path the timed stream takes (lone and
    # batched frames, the double re-run) has run once before the clock starts
    n_warm_pool = 16
    wrng = np.random.default_rng(4)
    warm_pool = make_pool(np.maximum(1, np.round(wrng.lognormal(math.log(15000), 0.6, n_warm_pool))),
                          np.random.SeedSequence(4).spawn(n_warm_pool))
    n_fr = int(args.serve_rate * args.serve_seconds)
    t = np.cumsum(rng.exponential(1.0 / args.serve_rate, n_fr))
    t_warm = np.cumsum(wrng.exponential(1.0 / args.serve_rate, max(8, int(args.serve_rate))))

    def stream(times, frames=pool):
        return [serve.Frame(i, float(times[i]), *frames[i % len(frames)][:2], frames[i % len(frames)][2])
                for i in range(len(times))]

    n_of = {i: pool[i % n_pool][0] for i in range(n_fr)}
    out = {"metric": "served frame latency and tracks/s (continuous batching)", "unit": "ms",
           "data": "synthetic", "n_gpus": 1,
           "config": {"workload": f"Poisson {args.serve_rate:g} frames/s for {args.serve_seconds:g} s, "
                                  f"lognormal tracks (median 15000, sigma 0.6), 50% fakes, "
                                  f"{n_pool} distinct frames cycled", "hbm_budget_gb": 32}}
    for name, prec, policy, slots in (("continuous_fp32", "fp32", "continuous", 2),
                                      ("static_fp64", "fp64", "static", 1)):
        # the consumer reads every frame's results (its matched tracks) and
        # keeps none of them, as the next stage of a readout chain would
        matched = [0]

        def consume(fid, r):
            matched[0] += int(np.count_nonzero(r["n_match"]))

        ex = serve.HipExecutor(P, prec, budget_bytes=32 << 30, n_slots=slots, on_result=consume)
        sched = serve.Scheduler(ex, policy, static_frames=8, static_timeout_s=0.02)
        sched.run(stream(t_warm, warm_pool))
        torch.cuda.synchronize()
        log(f"serving {n_fr} frames: {name}")
        matched[0] = 0
        done = sched.run(stream(t))
        out[name] = serve.summarize(done, n_of)
        out[name]["matched_tracks"] = matched[0]
        log(f"  {out[name]}")
        # saturation: every frame present at t = 0
        sat = sched.run(stream(np.zeros(min(n_fr, 400))))
        out[name]["saturation_tracks_per_s"] = serve.summarize(sat, n_of)["tracks_per_s"]
        ex.close()
    out["value"] = out["continuous_fp32"]["p99_ms"]
    out["higher_is_better"] = False
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c5_distortion_450k")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp32_cov64", "fp64"])
    ap.add_argument("--block-size", type=int, default=0)
    ap.add_argument("--search-lanes", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain FP64 comparator")
    ap.add_argument("--graph", action="store_true", help="replay bin + match as one captured graph")
    ap.add_argument("--separate", action="store_true",
                    help="time trd_load_tracklets + trd_match instead of the one trd_load_and_match call")
    ap.add_argument("--n-hyp", type=int, default=0,
                    help="hypotheses kept per layer (0: the single best candidate)")
    ap.add_argument("--chi2-penalty", type=float, default=None,
                    help="cost of a layer without a tracklet when --n-hyp > 0 (default chi2_max)")
    ap.add_argument("--persistent", action="store_true",
                    help="one-lane-per-track match as a persistent grid")
    ap.add_argument("--autotune", action="store_true", help="pick block size and lanes per track first")
    ap.add_argument("--serve", action="store_true", help="serving benchmark (Poisson frame stream)")
    ap.add_argument("--residuals", action="store_true", help="residual-map benchmark on the 450k batch")
    ap.add_argument("--realistic", action="store_true",
                    help="realistic detector: energy loss in every layer and the 522-chamber layout")
    ap.add_argument("--serve-rate", type=float, default=200.0)
    ap.add_argument("--serve-seconds", type=float, default=5.0)
    ap.add_argument("--serve-pool", type=int, default=48)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a 512 MiB elementwise copy first (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the path shards by "
                                   "time frame with no exchange between GPUs, and multi-GPU runs "
                                   "are not part of it", "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    from paper_2003_03174_amd import synth
    assert torch.cuda.is_available(), "bench needs a HIP device"
    if args.serve:
        serve_bench(args)
        return
    if args.residuals:
        residual_bench(args)
        return

    if args.calibrate_copy:
        # an elementwise kernel that reads 512 MiB and writes 512 MiB once
        src = torch.ones(128 * 1024 * 1024, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        log("calibration: 3 x (512 MiB read + 512 MiB written) by an elementwise add")
        del src, dst
    log(f"generating {args.workload}")
    if args.realistic:
        w = synth.generate(args.workload, params=synth.realistic_overrides())
    else:
        w = synth.load_workload(args.workload)
    if args.n_hyp:
        w = dict(w)
        w["params"] = dict(w["params"], n_hyp=args.n_hyp,
                           chi2_penalty=(args.chi2_penalty if args.chi2_penalty is not None
                                         else w["params"]["chi2_max"]))
    P = w["params"]
    n, ntk, ng = w["n_tracks"], w["n_tracklets"], w["n_groups"]
    n_cells = ng * 540 * P["n_rows"] * P["n_yb"] * P["n_db"]
    log(f"{n} tracks, {ntk} tracklets, {n_cells} cells; timing {args.precision}")
    tuned = None
    if args.autotune:
        from paper_2003_03174_amd import autotune, binding
        d = binding.device_inputs(synth.to_device_layout(w), args.precision)
        tuned = autotune.tune(P, d, ng, args.precision, use_cache=False)
        args.block_size, args.search_lanes = tuned["block_size"], tuned["search_lanes"]
        args.persistent = tuned["persistent"]
        w = dict(w, params=dict(P, **tuned["bins"]))
        P = w["params"]
        n_cells = ng * 540 * P["n_rows"] * P["n_yb"] * P["n_db"]
        log(f"autotuned: bins {tuned['bins']}, block {args.block_size}, lanes {args.search_lanes}, "
            f"persistent {args.persistent} ({tuned['ms']:.3f} ms)")
        del d
    from paper_2003_03174_amd import binding
    r = run_gpu(w, args.precision, args.steps, args.warmup, args.block_size, args.search_lanes,
                graph=args.graph, flags=binding.TRD_CFG_PERSISTENT if args.persistent else 0,
                fused=not args.separate)
    ms = r["wall_ms_per_step"]
    split = r["match_ms"] is not None
    match_avg = sum(r["match_ms"]) / len(r["match_ms"]) if split else None
    bin_avg = sum(r["bin_ms"]) / len(r["bin_ms"]) if split else None
    log(f"{ms:.3f} ms/step" + (f" (bin {bin_avg:.3f} ms, match {match_avg:.3f} ms)" if split else " (one graph)"))
    ab = match_alg_bytes(n, ntk, n_cells, args.precision)
    kms = r["kernel_ms"][-args.steps:]
    if not kms:
        raise RuntimeError("the match kernel recorded no durations")
    kernel_avg = sum(kms) / len(kms)
    achieved = ab / (kernel_avg * 1e-3) / 1e9
    traffic = profiled_traffic() if (args.workload == "c5_distortion_450k" and args.precision == "fp32"
                                     and not args.search_lanes > 1 and not args.persistent
                                     and not args.n_hyp and not args.realistic) else None
    line = {
        "metric": "matched tracks/s (6-layer Kalman)",
        "value": n / (ms * 1e-3),
        "unit": "tracks/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision != "fp64" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {n} seed tracks, {ntk} tracklets, {ng} group(s); "
                        + synth.describe(args.workload) + f"; {n_cells} cells"
                        + ("; realistic detector: Bethe energy loss of 1.2 g/cm^2 per layer, "
                           "522 of 540 chambers" if args.realistic else ""),
            "graph": bool(args.graph),
            "precision": args.precision,
            "block_size": args.block_size or 256,
            "search_lanes": args.search_lanes or 1,
            "persistent": bool(args.persistent),
            "n_hyp": args.n_hyp,
            "chi2_penalty": P.get("chi2_penalty") if args.n_hyp else None,
            "step": "bin all tracklets + match all tracks"
                    + (" (trd_load_tracklets + trd_match)" if args.separate else
                       " (trd_load_and_match: the seeds are ordered while the tracklets are binned)"),
        },
        "latency_ms": {"step_p50": pct(r["step_ms"], 50), "step_p99": pct(r["step_ms"], 99),
                       "bin_avg": bin_avg, "match_avg": match_avg, "match_kernel_avg": kernel_avg,
                       "steps_from": "events around each step, in a pass of as many steps after the timed ones",
                       "split_from": None if (args.separate or args.graph) else
                       "separate trd_load_tracklets + trd_match calls after the timed steps"},
        "tracks_ge2_matches_per_s": r["n_ge2"] / (ms * 1e-3),
        "refit": {"ms": sum(r["refit_ms"]) / len(r["refit_ms"]),
                  "tracks_per_s": n / (sum(r["refit_ms"]) / len(r["refit_ms"]) * 1e-3),
                  "what": "TRD-only refit of all matched tracks (one launch, after the timed steps)"},
        "fp64_fallback_tracks": r["n_fallback"],
        "autotune": {"bins": tuned["bins"], "bin_table": tuned["bin_table"], "shapes": tuned["table"]}
                    if tuned else None,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_match_beam" if args.n_hyp else "k_match", "alg_bytes_per_launch": ab,
                     "kernel_ms": kernel_avg},
        # what bounds k_match instead: its share of the VALU issue slots and
        # of active lanes per instruction, from the committed counter summary
        "valu": profiled_valu() if traffic is not None else None,
    }
    if line["valu"] is not None:
        v = line["valu"]
        line["roofline"]["binding"] = (f"VALU issue and lane divergence: {100 * v['issue_frac']:.0f} % of the "
                                       f"issue slots, {100 * v['lane_frac']:.0f} % of the lanes active; HBM "
                                       f"{100 * line['roofline']['frac']:.1f} % on algorithmic bytes")
    if not args.no_fp64 and args.precision != "fp64":
        log("timing the plain FP64 comparator")
        r64 = run_gpu(w, "fp64", max(3, args.steps // 2), 2)
        line["fp64_plain"] = {"value": n / (r64["wall_ms_per_step"] * 1e-3), "unit": "tracks/s",
                              "ms_per_step": r64["wall_ms_per_step"],
                              "match_avg_ms": sum(r64["match_ms"]) / len(r64["match_ms"])}
    if not args.no_cpu_baseline:
        log("timing the CPU oracle on a bounded sample")
        line["cpu_baseline"] = cpu_baseline(w, gpu=r["result"], prec=args.precision)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
