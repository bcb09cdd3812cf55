"""Continuous batching of time frames onto the matcher (serving loop).

Frames arrive over time (trigger-tagged tracklets and seed tracks of one
interaction group each; a track only sees its own frame's tracklets).  The
server keeps a FIFO of arrived frames and a fixed set of execution slots,
each a HIP stream with its own matcher context and device buffers reserved
once from the HBM budget.  Whenever a slot is free it takes every queued
frame that fits the slot's capacity (continuous policy) and launches one
bin + match over them as groups of one batch; batches on different slots
overlap on the device.  The static policy instead waits for a fixed number
of frames or a timeout.  A frame larger than a slot is rejected on its own;
the others are unaffected.

The scheduler is independent of the device: `Scheduler` drives any executor
with launch/poll/collect methods; `HipExecutor` is the device one.
"""
from __future__ import annotations

import gc
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Frame:
    fid: int
    arrival: float          # seconds from the start of the stream
    n_tracks: int
    n_tracklets: int
    data: dict = field(default=None, repr=False)   # host arrays (see frame_arrays)


@dataclass
class Done:
    fid: int
    arrival: float
    launched: float
    finished: float
    batch: int
    n_frames_in_batch: int
    device_ms: float = float("nan")
    rejected: str = ""

    @property
    def latency(self):
        return self.finished - self.arrival


class Scheduler:
    """Admission and batching policy, device-agnostic.

    executor: launch(frames) -> handle, poll(handle) -> bool (done),
    collect(handle) -> device_ms, n_slots, fits(frames) -> bool,
    frame_fits(frame) -> bool.
    policy: "continuous" or "static" (static_frames / static_timeout_s).
    """

    def __init__(self, executor, policy="continuous", static_frames=8, static_timeout_s=0.02,
                 clock=time.perf_counter, sleep=time.sleep, idle_gc=True):
        assert policy in ("continuous", "static")
        self.ex = executor
        self.policy = policy
        self.static_frames = static_frames
        self.static_timeout_s = static_timeout_s
        self.clock = clock
        self.sleep = sleep
        # A full collection of Python's cyclic garbage walks every tracked
        # object of the process (torch's alone are several hundred thousand)
        # and stalls the loop for milliseconds.  With idle_gc the automatic
        # collector is off while `run` serves; the two young generations are
        # collected only when the loop has nothing to do, and the previous
        # collector state comes back when `run` returns.
        self.idle_gc = idle_gc

    def _take(self, queue, now):
        """Frames for the next batch (FIFO prefix that fits), or []."""
        if not queue:
            return []
        if self.policy == "static":
            waited = now - queue[0].arrival
            if len(queue) < self.static_frames and waited < self.static_timeout_s:
                return []
        batch = []
        limit = self.static_frames if self.policy == "static" else None
        while queue and (limit is None or len(batch) < limit):
            cand = batch + [queue[0]]
            if not self.ex.fits(cand):
                break
            batch.append(queue.popleft())
        return batch

    def run(self, frames, realtime=True):
        """Serve `frames` (sorted by arrival).  Returns a list of Done."""
        if not self.idle_gc:
            return self._run(frames, realtime)
        was_enabled = gc.isenabled()
        gc.disable()
        try:
            return self._run(frames, realtime)
        finally:
            if was_enabled:
                gc.enable()

    def _collect_young(self):
        young, middle, _ = gc.get_count()
        th0, th1, _ = gc.get_threshold()
        if middle >= th1:
            gc.collect(1)
        elif young >= th0:
            gc.collect(0)

    def _run(self, frames, realtime):
        pending = deque(sorted(frames, key=lambda f: f.arrival))
        queue = deque()
        free = list(range(self.ex.n_slots))
        inflight = []          # (slot, handle, frames, launch_time, batch_no)
        done = []
        t0 = self.clock()
        sim_now = 0.0
        nbatch = 0
        while pending or queue or inflight:
            now = (self.clock() - t0) if realtime else sim_now
            if not realtime:
                self.ex.now = now
            while pending and pending[0].arrival <= now:
                f = pending.popleft()
                if not self.ex.frame_fits(f):
                    done.append(Done(f.fid, f.arrival, now, now, -1, 0, rejected="larger than a slot"))
                    continue
                queue.append(f)
            progressed = False
            for item in list(inflight):
                slot, h, fr, tl, bno = item
                if self.ex.poll(h):
                    t_end = (self.clock() - t0) if realtime else now
                    dev_ms = self.ex.collect(h)
                    for f in fr:
                        done.append(Done(f.fid, f.arrival, tl, t_end, bno, len(fr), dev_ms))
                    inflight.remove(item)
                    free.append(slot)
                    progressed = True
            while free and queue:
                batch = self._take(queue, now)
                if not batch:
                    break
                slot = free.pop(0)
                h = self.ex.launch(slot, batch)
                inflight.append((slot, h, batch, now, nbatch))
                nbatch += 1
                progressed = True
            if not progressed:
                if self.idle_gc:
                    self._collect_young()
                if realtime:
                    self.sleep(5e-5)
                else:
                    # advance simulated time to the next event
                    nxt = [pending[0].arrival] if pending else []
                    nxt += [self.ex.eta(h) for (_, h, _, _, _) in inflight] if inflight else []
                    if self.policy == "static" and queue:
                        nxt.append(queue[0].arrival + self.static_timeout_s)
                    sim_now = max(sim_now, min(nxt)) if nxt else sim_now + 1e-6
        return done


def summarize(done, n_tracks_of):
    """Latency percentiles (ms) and throughput of a served stream."""
    ok = [d for d in done if not d.rejected]
    lat = np.array([d.latency for d in ok]) * 1e3
    dev = np.array([d.device_ms for d in ok])
    span = max(d.finished for d in ok) - min(d.arrival for d in ok) if ok else float("nan")
    trk = sum(n_tracks_of[d.fid] for d in ok)
    return dict(
        frames=len(ok), rejected=len(done) - len(ok),
        p50_ms=float(np.percentile(lat, 50)) if ok else math.nan,
        p99_ms=float(np.percentile(lat, 99)) if ok else math.nan,
        mean_ms=float(lat.mean()) if ok else math.nan,
        device_p50_ms=float(np.nanpercentile(dev, 50)) if ok else math.nan,
        tracks_per_s=trk / span if ok and span > 0 else math.nan,
        batches=len({d.batch for d in ok}),
        mean_frames_per_batch=float(np.mean([d.n_frames_in_batch for d in ok])) if ok else math.nan,
    )


# ---------------------------------------------------------------------------
# device executor
# ---------------------------------------------------------------------------

IN_TRK = {"p": 5, "cov": 15, "x": 1, "sector": 1, "group": 1}
IN_TKL = {"y": 1, "z": 1, "dy": 1, "det_row": 1, "tgroup": 1}
OUT = {"idx": 6, "p": 5, "cov": 15, "x": 1, "sector": 1, "chi2": 1, "chi2_layer": 6, "n_match": 1,
       "status": 1}
INT_KEYS = {"sector", "group", "det_row", "tgroup", "idx", "n_match", "status"}
TKL_FLOAT32 = {"y", "z", "dy"}   # tracklet fields are float whatever the precision


def pack_layout(spec, n_of, float_bytes):
    """Byte layout of a batch's arrays packed into one buffer: key -> (offset,
    rows, n, kind) with kind "i" (int32), "f32" or "f" (the state's float of
    float_bytes), each array 256-byte aligned; and the total size.  One copy
    then moves a whole batch between host and device."""
    lay, off = {}, 0
    for k, rows in spec.items():
        kind = "i" if k in INT_KEYS else ("f32" if k in TKL_FLOAT32 else "f")
        es = 4 if kind != "f" else float_bytes
        n = n_of(k)
        lay[k] = (off, rows, n, kind)
        off += (rows * n * es + 255) // 256 * 256
    return lay, off


def _in_counts(n_tracks, n_tracklets):
    return lambda k: n_tracks if k in IN_TRK else n_tracklets


def frame_arrays(w, pinned=False):
    """Host arrays of one frame (single-group workload dict from synth).  With
    pinned=True the frame also carries its inputs packed in one page-locked
    buffer ("_blob", float state), as a readout that lands frames in DMA-able
    memory would hand them over: a batch of one such frame goes to the device
    in a single copy, without staging."""
    a = dict(
        p=np.ascontiguousarray(w["p"].astype(np.float32)),
        cov=np.ascontiguousarray(w["cov"].astype(np.float32)),
        x=np.ascontiguousarray(w["x"].astype(np.float32)),
        sector=np.ascontiguousarray(w["sector"].astype(np.int32)),
        y=np.ascontiguousarray(w["tkl_y"].astype(np.float32)),
        z=np.ascontiguousarray(w["tkl_z"].astype(np.float32)),
        dy=np.ascontiguousarray(w["tkl_dy"].astype(np.float32)),
        det_row=np.ascontiguousarray(w["tkl_det_row"].astype(np.uint32).view(np.int32)),
    )
    if pinned:
        import torch
        n, nt = a["x"].size, a["y"].size
        lay, size = pack_layout({**IN_TRK, **IN_TKL}, _in_counts(n, nt), 4)
        blob = torch.zeros(size, dtype=torch.uint8).pin_memory()
        buf = blob.numpy()
        for k, (off, rows, cnt, kind) in lay.items():
            if k in a:
                dst = buf[off:off + rows * cnt * 4].view(np.int32 if kind == "i" else np.float32)
                dst[:] = a[k].reshape(-1)
        a["_blob"] = blob
    return a


BYTES_PER_TRACK = 4 * (21 + 2) + 4 * (21 + 6 + 4 + 1 + 6)     # inputs + outputs (float)
BYTES_PER_TRACKLET = 4 * 5 + 40 + 8                          # inputs + binning buffers
BYTES_PER_CELL = 4 + 1


class HipExecutor:
    """n_slots streams, each with a matcher context and flat device / pinned
    host buffers sized from the HBM budget (slot capacity = budget / n_slots,
    at most max_batch_tracks tracks); every batch uses contiguous views of
    exactly its size."""

    IN_TRK, IN_TKL, OUT = IN_TRK, IN_TKL, OUT

    def __init__(self, params, precision="fp32", budget_bytes=32 << 30, n_slots=2,
                 tracklets_per_track=12.0, max_groups=256, device=0, block_size=0, search_lanes=0,
                 max_batch_tracks=2_000_000, on_result=None):
        """on_result(fid, arrays) receives each frame's results as they are
        collected; without it they accumulate in `results` until the caller
        takes them out, which a long-running server must do (every frame
        holds about 160 bytes per track)."""
        import torch

        from . import binding as B
        self.torch = torch
        self.params = params
        self.precision = precision
        self.n_slots = n_slots
        self.max_groups = max_groups
        cells_per_group = 540 * params["n_rows"] * params["n_db"] * params["n_yb"]
        per_slot = budget_bytes // n_slots - max_groups * cells_per_group * BYTES_PER_CELL
        if per_slot <= 0:
            raise ValueError("HBM budget too small for the cell tables of one slot")
        per_track = BYTES_PER_TRACK + tracklets_per_track * BYTES_PER_TRACKLET
        self.cap_tracks = int(min(per_slot // per_track, max_batch_tracks))
        self.cap_tracklets = int(self.cap_tracks * tracklets_per_track)
        dev = torch.device("cuda", device)
        self.float_bytes = 8 if precision == "fp64" else 4
        self.dtypes = {"i": torch.int32, "f32": torch.float32,
                       "f": torch.float64 if precision == "fp64" else torch.float32}
        T, K = self.cap_tracks, self.cap_tracklets
        # each slot: one device and one page-locked buffer for the batch's
        # inputs, the same for its outputs (a batch moves in one copy each way)
        _, in_bytes = pack_layout({**self.IN_TRK, **self.IN_TKL}, _in_counts(T, K), self.float_bytes)
        _, out_bytes = pack_layout(self.OUT, lambda k: T, self.float_bytes)
        self.slots = []
        for _ in range(n_slots):
            m = B.Matcher(params, precision, device=device, block_size=block_size,
                          search_lanes=search_lanes)
            m.reserve(K, max_groups, T)
            self.slots.append(dict(
                m=m, stream=torch.cuda.Stream(device=dev),
                din=torch.empty(in_bytes, dtype=torch.uint8, device=dev),
                hin=torch.empty(in_bytes, dtype=torch.uint8, pin_memory=True),
                dout=torch.empty(out_bytes, dtype=torch.uint8, device=dev),
                hout=torch.empty(out_bytes, dtype=torch.uint8, pin_memory=True)))
        self.results = {}
        self.on_result = on_result

    # -- capacity ------------------------------------------------------------
    def frame_fits(self, f):
        return f.n_tracks <= self.cap_tracks and f.n_tracklets <= self.cap_tracklets

    def fits(self, frames):
        return (len(frames) <= self.max_groups and
                sum(f.n_tracks for f in frames) <= self.cap_tracks and
                sum(f.n_tracklets for f in frames) <= self.cap_tracklets)

    def _views(self, blob, lay):
        """Typed [rows][n] (or [n]) views of a packed buffer."""
        out = {}
        for k, (off, rows, n, kind) in lay.items():
            dt = self.dtypes[kind]
            es = 8 if dt == self.torch.float64 else 4
            v = blob[off:off + rows * n * es].view(dt)
            out[k] = v.view(rows, n) if rows > 1 else v
        return out

    # -- execution -----------------------------------------------------------
    def launch(self, slot, frames):
        torch = self.torch
        S = self.slots[slot]
        s, m = S["stream"], S["m"]
        ntr = sum(f.n_tracks for f in frames)
        ntk = sum(f.n_tracklets for f in frames)
        lay_in, nb_in = pack_layout({**self.IN_TRK, **self.IN_TKL}, _in_counts(ntr, ntk), self.float_bytes)
        lay_out, nb_out = pack_layout(self.OUT, lambda k: ntr, self.float_bytes)
        # a single frame that arrived packed in page-locked memory goes to the
        # device as it is; otherwise the batch is packed into the slot's
        # pinned buffer (free: the slot is idle)
        blob = frames[0].data.get("_blob") if len(frames) == 1 else None
        src = blob if (blob is not None and self.float_bytes == 4) else None
        if src is None:
            hv = self._views(S["hin"], lay_in)
            for k, v in hv.items():
                if k == "group":
                    parts = [np.full(f.n_tracks, i, np.int32) for i, f in enumerate(frames)]
                elif k == "tgroup":
                    parts = [np.full(f.n_tracklets, i, np.int32) for i, f in enumerate(frames)]
                else:
                    parts = [np.asarray(f.data[k]) for f in frames]
                np.concatenate(parts, axis=-1, out=v.numpy())
            src = S["hin"]
        ev0, ev1, done = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True),
                          torch.cuda.Event())
        with torch.cuda.stream(s):
            S["din"][:nb_in].copy_(src[:nb_in], non_blocking=True)
            dv = self._views(S["din"], lay_in)
            ev0.record(s)
            out = self._views(S["dout"], lay_out)
            m.load_and_match(dv["y"], dv["z"], dv["dy"], dv["det_row"], dv["tgroup"], len(frames), dv["p"],
                             dv["cov"], dv["x"], dv["sector"], tgroup=dv["group"], out=out, stream=s)
            ev1.record(s)
            S["hout"][:nb_out].copy_(S["dout"][:nb_out], non_blocking=True)
            done.record(s)
        return dict(frames=frames, done=done, ev=(ev0, ev1), host=self._views(S["hout"], lay_out))

    def poll(self, h):
        return h["done"].query()

    def collect(self, h):
        """Per-frame results with frame-local tracklet indices."""
        h["done"].synchronize()
        off, toff = 0, 0
        for f in h["frames"]:
            sl = slice(off, off + f.n_tracks)
            r = {k: v.numpy()[..., sl].copy() for k, v in h["host"].items()}
            r["idx"] = np.where(r["idx"] >= 0, r["idx"] - toff, -1).astype(np.int32)
            if self.on_result is not None:
                self.on_result(f.fid, r)
            else:
                self.results[f.fid] = r
            off += f.n_tracks
            toff += f.n_tracklets
        ms = h["ev"][0].elapsed_time(h["ev"][1])
        h.clear()
        return ms

    def eta(self, h):
        return 0.0

    def close(self):
        for S in self.slots:
            S["m"].close()


class FakeExecutor:
    """Device-free executor for testing the scheduler: a batch completes a
    fixed time per track after its launch (simulated clock)."""

    def __init__(self, cap_tracks, cap_tracklets, n_slots=2, s_per_track=1e-7, s_launch=2e-5,
                 max_groups=256):
        self.cap_tracks, self.cap_tracklets = cap_tracks, cap_tracklets
        self.n_slots, self.s_per_track, self.s_launch = n_slots, s_per_track, s_launch
        self.max_groups = max_groups
        self.now = 0.0
        self.launched = []

    frame_fits = HipExecutor.frame_fits
    fits = HipExecutor.fits

    def launch(self, slot, frames):
        t_done = self.now + self.s_launch + self.s_per_track * sum(f.n_tracks for f in frames)
        self.launched.append((slot, [f.fid for f in frames]))
        return dict(t=t_done, slot=slot)

    def poll(self, h):
        return self.now >= h["t"]

    def collect(self, h):
        return (h["t"] - self.now) * 1e3

    def eta(self, h):
        return h["t"]
