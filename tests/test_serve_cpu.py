"""Scheduler of the serving loop on a simulated device (no GPU)."""
import gc
import weakref

import numpy as np

from paper_2003_03174_amd.serve import FakeExecutor, Frame, Scheduler, summarize


def _stream(n, rate, seed=0, median=15000, sigma=0.6, tpt=9):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, n))
    sizes = np.maximum(1, np.round(rng.lognormal(np.log(median), sigma, n))).astype(int)
    return [Frame(i, float(t[i]), int(sizes[i]), int(sizes[i] * tpt)) for i in range(n)]


def test_light_load_serves_frames_alone():
    ex = FakeExecutor(cap_tracks=200000, cap_tracklets=2000000, s_per_track=1e-8)
    frames = _stream(50, rate=20.0)
    done = Scheduler(ex, "continuous").run(frames, realtime=False)
    assert len(done) == 50 and not any(d.rejected for d in done)
    assert all(d.n_frames_in_batch == 1 for d in done)
    assert all(d.latency >= 0 for d in done)


def test_heavy_load_batches_continuously_and_overlaps():
    ex = FakeExecutor(cap_tracks=100000, cap_tracklets=900000, n_slots=2, s_per_track=2e-7)
    frames = _stream(300, rate=400.0)
    done = Scheduler(ex, "continuous").run(frames, realtime=False)
    assert len(done) == 300
    s = summarize(done, {f.fid: f.n_tracks for f in frames})
    assert s["mean_frames_per_batch"] > 1.2
    assert max(d.n_frames_in_batch for d in done) >= 3
    # never more than the slot capacity per batch, FIFO across batches
    by_batch = {}
    for d in done:
        by_batch.setdefault(d.batch, []).append(d)
    for b, ds in by_batch.items():
        assert sum(next(f for f in frames if f.fid == d.fid).n_tracks for d in ds) <= 100000
    order = sorted(done, key=lambda d: d.fid)
    assert all(order[i].batch <= order[i + 1].batch for i in range(len(order) - 1))
    # both slots were busy at the same time at some point
    spans = sorted({(d.launched, d.finished) for d in done})
    assert any(spans[i + 1][0] < spans[i][1] for i in range(len(spans) - 1))


def test_oversize_frame_is_rejected_alone():
    ex = FakeExecutor(cap_tracks=10000, cap_tracklets=90000)
    frames = [Frame(0, 0.0, 5000, 45000), Frame(1, 0.001, 20000, 180000), Frame(2, 0.002, 3000, 27000)]
    done = {d.fid: d for d in Scheduler(ex).run(frames, realtime=False)}
    assert done[1].rejected and not done[0].rejected and not done[2].rejected


def test_static_policy_waits_for_count_or_timeout():
    ex = FakeExecutor(cap_tracks=10 ** 7, cap_tracklets=10 ** 8, n_slots=1, s_per_track=1e-9)
    frames = [Frame(i, 0.001 * i, 1000, 9000) for i in range(10)]
    done = Scheduler(ex, "static", static_frames=4, static_timeout_s=0.05).run(frames, realtime=False)
    sizes = sorted({d.batch: d.n_frames_in_batch for d in done}.values(), reverse=True)
    assert sizes[:2] == [4, 4]
    last = [d for d in done if d.n_frames_in_batch == 2]
    # the timeout runs from the oldest queued frame (arrival 0.008 s)
    assert len(last) == 2 and all(abs(d.launched - (0.008 + 0.05)) < 1e-9 for d in last)


class _Cycle:
    def __init__(self):
        self.me = self


class _GarbageExecutor(FakeExecutor):
    """Leaves cyclic garbage behind at every launch, as host code does."""

    def __init__(self, *a, **k):
        super().__init__(*a, **k)
        self.refs = []

    def launch(self, slot, frames):
        for _ in range(400):
            c = _Cycle()
            self.refs.append(weakref.ref(c))
        return super().launch(slot, frames)


def test_idle_collection_frees_young_garbage_and_restores_the_collector():
    for enabled in (True, False):
        ex = _GarbageExecutor(cap_tracks=200000, cap_tracklets=2000000, s_per_track=1e-8)
        (gc.enable if enabled else gc.disable)()
        try:
            full_before = gc.get_stats()[2]["collections"]
            done = Scheduler(ex, "continuous").run(_stream(60, rate=20.0), realtime=False)
            full_after = gc.get_stats()[2]["collections"]
            assert gc.isenabled() == enabled
        finally:
            gc.enable()
        assert len(done) == 60
        # no full collection while serving; the cycles died in idle time
        assert full_after == full_before
        dead = sum(r() is None for r in ex.refs)
        assert dead >= 0.9 * len(ex.refs)


def test_idle_collection_off_leaves_the_collector_alone():
    ex = FakeExecutor(cap_tracks=200000, cap_tracklets=2000000, s_per_track=1e-8)
    gc.disable()
    try:
        Scheduler(ex, "continuous", idle_gc=False).run(_stream(10, rate=20.0), realtime=False)
        assert not gc.isenabled()
    finally:
        gc.enable()
