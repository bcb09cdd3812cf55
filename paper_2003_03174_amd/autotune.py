"""Autotuner for the matcher's launch shape and tracklet cells.

Times one bin + match step on the device at hand and keeps the fastest, in
two stages:
  1. the cell geometry: y and dy bin widths over the same y and dy spans
     (the candidate set is the same for every geometry, binned and
     brute-force search agree; only the time differs), with the default
     launch shape;
  2. with that geometry, each (workgroup size, lanes per track) pair, and
     the persistent grid against the plain one (one lane per track).
Tracks per wavefront in the road scan are 64 / lanes.  Results are cached per
device name and workload signature in a JSON file.
"""
from __future__ import annotations

import hashlib
import json
import os
import time

from . import binding as B

DEFAULT_SHAPES = ((256, 1), (256, 4), (256, 8), (256, 16), (128, 4), (128, 8), (64, 4), (64, 8))
# bin widths tried (cm): each keeps the workload's y span n_yb * y_bin_w and
# dy span n_db * dy_bin_w
Y_WIDTHS = (4.0, 8.0, 16.0)
DY_WIDTHS = (0.125, 0.25, 0.5)


def bin_geometries(params, y_widths=Y_WIDTHS, dy_widths=DY_WIDTHS):
    """Cell geometries with the workload's y span and its dy span (8 cm,
    +-4 cm, when it does not bin dy yet): each y width with no dy bins and
    with each dy width that divides the span into a whole number of bins."""
    ys = params["n_yb"] * params["y_bin_w"]
    ds = params["n_db"] * params["dy_bin_w"] if params["n_db"] > 1 else 8.0
    dys = [(params["dy_bin_w"] if params["n_db"] == 1 else ds, 1)]
    for wd in dy_widths:
        nd = ds / wd
        if nd >= 1 and nd == int(nd) and nd <= 4096:
            dys.append((wd, int(nd)))
    out = []
    for wy in y_widths:
        ny = ys / wy
        if not (ny >= 1 and ny == int(ny) and ny <= 4096):
            continue
        for wd, nd in dys:
            out.append(dict(y_bin_w=wy, n_yb=int(ny), dy_bin_w=wd, n_db=nd))
    return out


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


def _time_step(params, d, n_groups, precision, bs, lanes, flags, reps):
    import torch
    n = int(d["x"].numel())
    stream = torch.cuda.current_stream()
    m = B.Matcher(params, precision, block_size=bs, search_lanes=lanes, flags=flags)
    m.reserve(int(d["y"].numel()), n_groups, n)
    out = m.alloc_results(n, chi2_layer=False)
    ts = []
    for r in range(reps + 1):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        m.load_and_match(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], n_groups, d["p"], d["cov"], d["x"],
                         d["sector"], tgroup=d["group"], out=out)
        e1.record(stream)
        torch.cuda.synchronize()
        if r:
            ts.append(e0.elapsed_time(e1))
    m.close()
    ts.sort()
    return ts[len(ts) // 2]


def tune(params, d, n_groups, precision="fp32", shapes=DEFAULT_SHAPES, reps=5, use_cache=True,
         cache_path=None, geometries=None, persistent=(False, True)):
    """d: device tensors as from binding.device_inputs().  geometries: cell
    geometries to try (default: bin_geometries(params); pass [] to keep the
    workload's).  Returns {"block_size", "search_lanes", "persistent",
    "bins": {y_bin_w, n_yb, dy_bin_w, n_db}, "ms", "table": [(block, lanes,
    persistent, ms), ...], "bin_table": [(y_bin_w, dy_bin_w, ms), ...]}."""
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
    # stage 1: the cell geometry, default launch shape
    geos = bin_geometries(params) if geometries is None else list(geometries)
    # (cell offsets are 4 bytes a cell and written at every load: at most 2^26 cells)
    geos = [gq for gq in geos if n_groups * 540 * params["n_rows"] * gq["n_yb"] * gq["n_db"] <= 1 << 26]
    own = {k: params[k] for k in ("y_bin_w", "n_yb", "dy_bin_w", "n_db")}
    if own not in geos:
        geos.append(own)
    bin_table = []
    for gq in geos:
        bin_table.append((gq["y_bin_w"], gq["dy_bin_w"],
                          _time_step(dict(params, **gq), d, n_groups, precision, 256, 1, 0, reps)))
    by, bd, _ = min(bin_table, key=lambda t: t[2])
    bins = next(gq for gq in geos if gq["y_bin_w"] == by and gq["dy_bin_w"] == bd)
    P = dict(params, **bins)
    # stage 2: launch shape and grid kind with that geometry
    table = []
    for bs, lanes in shapes:
        for pers in persistent:
            if pers and lanes > 1:
                continue
            table.append((bs, lanes, bool(pers),
                          _time_step(P, d, n_groups, precision, bs, lanes, B.TRD_CFG_PERSISTENT if pers else 0,
                                     reps)))
    best = min(table, key=lambda t: t[3])
    res = {"block_size": best[0], "search_lanes": best[1], "persistent": best[2], "bins": bins, "ms": best[3],
           "table": table, "bin_table": bin_table, "device": dev, "tuned_at": time.time()}
    if use_cache:
        cache[key] = res
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            json.dump(cache, open(path, "w"), indent=1)
        except OSError:
            pass
    return res
