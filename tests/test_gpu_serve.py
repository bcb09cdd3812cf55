"""Serving loop on the device: each frame's result is the same alone and in
a continuously batched, overlapping stream."""
import numpy as np
import pytest

from paper_2003_03174_amd import synth
from paper_2003_03174_amd.serve import Frame, HipExecutor, Scheduler, frame_arrays, summarize

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def test_results_identical_alone_and_in_the_mix():
    P = synth.default_params()
    rng = np.random.default_rng(4)
    n = 24
    sizes = np.maximum(50, np.round(rng.lognormal(np.log(2000), 0.6, n))).astype(int)
    ss = np.random.SeedSequence(44).spawn(n)
    frames = []
    for i in range(n):
        g = synth.generate_group(np.random.default_rng(ss[i]), P, int(sizes[i]), fake_ratio=0.5,
                                 ineff_frac=0.1)
        w = synth._concat_groups([g], P)
        # every other frame in page-locked memory: alone it goes to the device
        # without staging, in a batch it is staged like the others
        data = frame_arrays(w, pinned=i % 2 == 0)
        frames.append(Frame(i, 0.0005 * i, w["n_tracks"], w["n_tracklets"], data))
    # results of the mix go to a consumer, those of the lone runs stay in
    # the executor's store
    mixed = {}
    ex = HipExecutor(P, "fp32", budget_bytes=4 << 30, n_slots=2, on_result=mixed.__setitem__)
    done = Scheduler(ex, "continuous").run(frames)
    assert not ex.results and sorted(mixed) == list(range(n))
    ex.on_result = None
    st = summarize(done, {f.fid: f.n_tracks for f in frames})
    print(st)
    assert st["frames"] == n and st["batches"] < n  # some batches hold several frames
    alone = {}
    for f in frames:
        ex.results.clear()
        Scheduler(ex, "continuous").run([Frame(f.fid, 0.0, f.n_tracks, f.n_tracklets, f.data)])
        alone[f.fid] = ex.results[f.fid]
    ex.close()
    for fid in alone:
        for k in alone[fid]:
            assert np.array_equal(alone[fid][k], mixed[fid][k], equal_nan=True), (fid, k)
