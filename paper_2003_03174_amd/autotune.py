"""Launch-shape autotuner for the matcher.

Times one bin + match step for each (workgroup size, lanes per track) pair on
the device at hand and keeps the fastest.  Tracks per wavefront in the road
scan are 64 / lanes.  Results are cached per device name and workload
signature in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import binding as B

DEFAULT_SHAPES = ((256, 1), (256, 4), (256, 8), (256, 16), (128, 4), (128, 8), (64, 4), (64, 8))


def _cache_path():
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "trd_mi355x", "launch_shapes.json")


def signature(params, n_tracks, n_tracklets, n_groups, precision):
    """Workload signature: binning geometry and the sizes rounded to 2x."""
    def bucket(v):
        return 0 if v <= 0 else int(v).bit_length()
    geo = (params["n_yb"], params["y_bin_w"], params["n_db"], params["dy_bin_w"],
           round(params["n_sigma_road"], 6), precision, bucket(n_tracks), bucket(n_tracklets),
           bucket(n_groups))
    return hashlib.sha1(repr(geo).encode()).hexdigest()[:16]


def tune(params, d, n_groups, precision="fp32", shapes=DEFAULT_SHAPES, reps=5, use_cache=True,
         cache_path=None):
    """d: device tensors as from binding.device_inputs().  Returns
    {"block_size", "search_lanes", "ms", "table": [(block, lanes, ms), ...]}."""
    import torch
    path = cache_path or _cache_path()
    dev = torch.cuda.get_device_name(0)
    n = int(d["x"].numel())
    sig = signature(params, n, int(d["y"].numel()), n_groups, precision)
    key = f"{dev}|{sig}"
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            cache = json.load(open(path))
        except (OSError, ValueError):
            cache = {}
        if key in cache:
            return cache[key]
    table = []
    stream = torch.cuda.current_stream()
    for bs, lanes in shapes:
        m = B.Matcher(params, precision, block_size=bs, search_lanes=lanes)
        m.reserve(int(d["y"].numel()), n_groups, n)
        out = m.alloc_results(n, chi2_layer=False)
        ts = []
        for r in range(reps + 1):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], n_groups)
            m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"], out=out)
            e1.record(stream)
            torch.cuda.synchronize()
            if r:
                ts.append(e0.elapsed_time(e1))
        m.close()
        ts.sort()
        table.append((bs, lanes, ts[len(ts) // 2]))
    best = min(table, key=lambda t: t[2])
    res = {"block_size": best[0], "search_lanes": best[1], "ms": best[2], "table": table,
           "device": dev, "tuned_at": time.time()}
    if use_cache:
        cache[key] = res
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return res
