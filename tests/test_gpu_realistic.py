"""The realistic detector model on the HIP path against the FP64 oracle,
through the C ABI: energy loss in every layer (matching outward, refit
inward), the 522-chamber layout (tracklets of empty slots dropped at load,
no hypothesis penalty in them), and tracks stopped by their energy loss."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
from tests import parity_util as pu

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

REAL = dict(eloss_xrho=1.2, eloss_za=0.53, eloss_i=70e-9)
_cache = {}


def workload(key, n, seed, fake_ratio=0.5, ineff=0.1, **params):
    if key not in _cache:
        P = dict(REAL, absent=synth.absent_522())
        P.update(params)
        _cache[key] = synth.generate(n_tracks=n, seed=seed, fake_ratio=fake_ratio, ineff_frac=ineff,
                                     params=P)
    return _cache[key]


def run(w, P, prec, planted=0):
    lay = synth.to_device_layout(w)
    d = B.device_inputs(lay, prec)
    y, z, dy, dr, tg = d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"]
    if planted:
        # tracklets in the empty slots: the load must drop them
        rng = np.random.default_rng(3)
        bad = np.nonzero(np.asarray(P["absent"]))[0]
        det = rng.choice(bad, planted)
        dev = y.device
        y = torch.cat([y, torch.from_numpy(rng.uniform(-30, 30, planted).astype(np.float32)).to(dev)])
        z = torch.cat([z, torch.from_numpy(rng.uniform(-60, 60, planted).astype(np.float32)).to(dev)])
        dy = torch.cat([dy, torch.from_numpy(rng.uniform(-1, 1, planted).astype(np.float32)).to(dev)])
        drw = ((det << 5) | rng.integers(0, 18, planted)).astype(np.uint32).view(np.int32)
        dr = torch.cat([dr, torch.from_numpy(drw).to(dev)])
        tg = torch.cat([tg, torch.zeros(planted, dtype=tg.dtype, device=dev)])
    m = B.Matcher(P, prec)
    m.load(y, z, dy, dr, tg, w["n_groups"])
    out = pu.to_numpy(m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"]))
    off, _ = m.binning()
    torch.cuda.synchronize()
    out["n_valid"] = int(off[-1].item())
    m.close()
    return out


@pytest.mark.parametrize("prec", ["fp64", "fp32_cov64", "fp32"])
def test_energy_loss_and_empty_slots(prec):
    w = workload("frame", 4000, 61)
    P = w["params"]
    got = run(w, P, prec, planted=300)
    # the 300 planted tracklets are gone; nothing of the generator's sits in an empty slot
    assert got["n_valid"] == w["n_tracklets"]
    ref = O.match(P, w, threads=0, margins=pu.MARGINS[prec])
    rep = pu.compare(ref, got, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()


def test_energy_loss_changes_the_answer():
    """The loss is really applied on the GPU: the same tracks matched without
    it end with a different momentum."""
    w = workload("frame", 4000, 61)
    P = w["params"]
    a = run(w, P, "fp64")
    Q = dict(P)
    Q["eloss_xrho"] = 0.0
    b = run(w, Q, "fp64")
    ok = (a["status"] == 0) & (b["status"] == 0) & (a["n_match"] == 6)
    rel = np.abs(a["p"][4, ok] / b["p"][4, ok] - 1.0)
    assert np.median(rel) > 1e-3


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_stopped_tracks(prec):
    """A thick layer stops the slow tracks: the same ones, at the same layer,
    as the oracle."""
    w = workload("thick", 2000, 62, eloss_xrho=40.0)
    P = w["params"]
    got = run(w, P, prec)
    ref = O.match(P, w, threads=0, margins=pu.MARGINS[prec])
    assert np.any(ref["status"] & O.ST_STOPPED)
    # 40 g/cm^2 per layer takes a large share of a slow track's kinetic
    # energy at every layer, and each loss multiplies the relative rounding
    # of the momentum by E_kin before / E_kin after; over six layers that
    # brings the float path to a few 1e-5 on q/pT (the double path keeps 1e-12)
    loose = 1e-4 if prec != "fp64" else None
    rep = pu.compare(ref, got, prec, state_tol_max=loose, q999_tol=loose)
    print(rep.summary())
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("n_hyp", [1, 2, 4])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_hypotheses_skip_no_penalty_in_empty_slots(prec, n_hyp):
    """The middle stack empty everywhere, so many hypotheses cross an empty
    slot; penalty 3 so that the rule decides between hypotheses."""
    ab = np.zeros(540, np.uint8)
    for sec in range(18):
        for l in range(6):
            ab[sec * 30 + 12 + l] = 1
    w = workload("beam", 3000, 63, absent=ab)
    P = dict(w["params"])
    P.update(n_hyp=n_hyp, chi2_penalty=3.0)
    got = run(w, P, prec)
    ref = O.match(P, w, threads=0, margins=pu.BEAM_MARGINS[prec])
    rep = pu.compare(ref, got, prec, max_flag_share=pu.MAX_FLAG_SHARE_BEAM)
    print(rep.summary())
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_refit_restores_the_energy_inward(prec):
    w = workload("frame", 4000, 61)
    P = w["params"]
    d = B.device_inputs(synth.to_device_layout(w), prec)
    m = B.Matcher(P, prec)
    m.load(d["y"], d["z"], d["dy"], d["det_row"], d["tgroup"], w["n_groups"])
    mo = m.match(d["p"], d["cov"], d["x"], d["sector"], d["group"])
    r = m.refit(mo, d["y"], d["z"], d["det_row"])
    torch.cuda.synchronize()
    matched = {k: mo[k].cpu().numpy() for k in ("p", "x", "sector", "idx")}
    got = {k: v.cpu().numpy() for k, v in r.items()}
    m.close()
    ref = O.refit(P, matched, matched["idx"], w)
    st = got["status"].astype(np.int64) & ~pu.GPU_ONLY_BITS
    assert np.array_equal(st, ref["status"].astype(np.int64))
    assert np.array_equal(got["n_used"], ref["n_used"])
    ok = (ref["status"] & 32) == 0
    dlt = np.abs(got["p"][:, ok].astype(np.float64) - ref["p"][:, ok])
    if prec == "fp64":
        e = dlt / np.maximum(np.abs(ref["p"][:, ok]), pu.FLOORS[:, None])
        assert e.max() <= pu.STATE_TOL["fp64"], e.max(axis=1)
    else:
        e = dlt / np.sqrt(ref["cov"][list(pu.DIAG)][:, ok])
        assert e.max() <= 1e-3, e.max(axis=1)


def test_detector_model_full_size_sampled():
    """The 450k batch with the detector model, as `bench.py --realistic` times
    it: 1,500 sampled tracks against the oracle."""
    w = synth.generate("c5_distortion_450k", params=synth.realistic_overrides())
    P = w["params"]
    got = run(w, P, "fp32")
    assert got["n_valid"] == w["n_tracklets"]
    sel = np.sort(np.random.default_rng(4).choice(w["n_tracks"], 1500, replace=False))
    ref = O.match(P, w, threads=0, margins=pu.MARGINS["fp32"], track_slice=sel)
    rep = pu.compare(ref, got, "fp32", sel=sel)
    print(rep.summary())
    assert rep.ok, rep.summary()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_near_infinite_momentum_loses_nothing(prec):
    """Seeds with |q/pT| = 1e-25 (a float square underflows): straight tracks
    that lose no measurable energy and are never stopped."""
    w = dict(workload("frame", 4000, 61))
    p = w["p"].copy()
    p[4, :40] = np.where(p[4, :40] < 0, -1e-25, 1e-25)
    w["p"] = p
    P = w["params"]
    got = run(w, P, prec)
    ref = O.match(P, w, threads=0, margins=pu.MARGINS[prec])
    assert not np.any(ref["status"][:40] & O.ST_STOPPED)
    assert not np.any(got["status"][:40] & O.ST_STOPPED)
    rep = pu.compare(ref, got, prec)
    print(rep.summary())
    assert rep.ok, rep.summary()
