"""Pins of the oracle's TRD-only refit (Sect. 2, step 3: refits from the outer
detectors with the TPC information ignored).

- noise-free tracklets, start at the truth: the inward propagation and the
  sector turns land on the generator's closed-form crossing of layer 0;
- noise-free tracklets, start displaced by many sigma of the TPC seed: the
  updates pull the state back to the truth (linearisation error only);
- with noise and scattering: pulls of all five parameters against the truth
  have mean 0 and RMS 1 (also with tilted pads); the chi2 sum has the mean of
  2m - 5 degrees of freedom under a flat start;
- the start state hardly matters (the TPC information is dropped);
- tracks with too few tracklets are copied with REFIT_FEW.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import synth

FLAT = (100.0, 1e4, 1.0, 1.0, 100.0)


def _frame(seed, n, **kw):
    P = synth.default_params(**kw.pop("params", {}))
    g = synth.generate_group(np.random.default_rng(seed), P, n, fake_ratio=0.0, ineff_frac=0.0, **kw)
    return P, synth._concat_groups([g], P)


def _truth0(w):
    T = w["truth"]
    return np.stack([T["y"][0], T["z"][0], T["snp"][0], T["tgl"][0], T["qpt"][0]]), T["sec"][0]


def _refit(P, m, w, p=None, cov=None):
    Q = dict(P)
    if cov is not None:
        Q["refit_cov"] = cov
    tr = dict(p=m["p"] if p is None else p, x=m["x"], sector=m["sector"])
    return O.refit(Q, tr, m["idx"], w)


def test_noise_free_from_the_truth_lands_on_the_crossing():
    P, w = _frame(7, 400, noise_free=True, ms=False)
    m = O.match(P, w, threads=0)
    r = _refit(P, m, w, cov=FLAT)
    truth, sec0 = _truth0(w)
    sel = (r["status"] == 0) & (r["n_used"] == 6) & (r["sector"] == sec0)
    assert sel.sum() > 350
    assert np.all(r["x"][sel] == P["x_layer"][0])
    err = np.abs(r["p"][:, sel] - truth[:, sel]).max(axis=1)
    assert np.all(err < 1e-9), err


def test_noise_free_from_a_displaced_start_returns_to_the_truth():
    P, w = _frame(7, 400, noise_free=True, ms=False)
    m = O.match(P, w, threads=0)
    p = m["p"].copy()
    p += np.array([0.2, 2.0, 2e-3, 2e-3, 0.05])[:, None]
    r = _refit(P, m, w, p=p, cov=FLAT)
    truth, sec0 = _truth0(w)
    sel = (r["status"] == 0) & (r["n_used"] == 6) & (r["sector"] == sec0)
    err = np.abs(r["p"][:, sel] - truth[:, sel]).max(axis=1)
    # second-order (linearisation) error of one pass; the displacement is
    # 2000x this in y and 100x in q/pT
    assert np.all(err < np.array([1e-4, 4e-3, 5e-5, 2e-4, 5e-3])), err


@pytest.mark.parametrize("tilt", [False, True])
def test_pulls_against_the_truth(tilt):
    params = dict(tilt=synth.tilt_pm2deg()) if tilt else {}
    P, w = _frame(11, 3000, params=params)
    m = O.match(P, w, threads=0)
    r = _refit(P, m, w, cov=FLAT)
    truth, sec0 = _truth0(w)
    sel = (r["status"] == 0) & (r["n_used"] == 6) & (r["sector"] == sec0) & (m["status"] == 0)
    assert sel.sum() > 2000
    diag = (0, 5, 9, 12, 14)
    pull = (r["p"][:, sel] - truth[:, sel]) / np.sqrt(r["cov"][list(diag)][:, sel])
    mean, rms = pull.mean(axis=1), pull.std(axis=1)
    assert np.all(np.abs(mean) < 0.1), mean
    assert np.all(np.abs(rms - 1.0) < 0.06), rms


@pytest.mark.parametrize("tilt", [False, True])
def test_chi2_sum_has_2m_minus_5_degrees_of_freedom(tilt):
    # with tilted pads the y and z residuals are strongly correlated
    params = dict(tilt=synth.tilt_pm2deg()) if tilt else {}
    P, w = _frame(13, 4000, params=params)
    m = O.match(P, w, threads=0)
    r = _refit(P, m, w, cov=FLAT)
    sel = (r["status"] == 0) & (r["n_used"] == 6)
    c = r["chi2"][sel]
    dof = 2 * 6 - 5
    assert abs(c.mean() - dof) < 3 * np.sqrt(2 * dof / c.size) + 0.1, c.mean()


def test_the_start_state_is_not_used():
    P, w = _frame(17, 1000)
    m = O.match(P, w, threads=0)
    a = _refit(P, m, w)
    p = m["p"].copy()
    p += np.array([0.1, 0.5, 1e-3, 1e-3, 0.02])[:, None]
    b = _refit(P, m, w, p=p)
    sel = (a["status"] == 0) & (b["status"] == 0) & (a["n_used"] == 6)
    diag = (0, 5, 9, 12, 14)
    sig = np.sqrt(a["cov"][list(diag)][:, sel])
    shift = np.abs(a["p"][:, sel] - b["p"][:, sel]) / sig
    assert np.all(shift.max(axis=1) < 0.1), shift.max(axis=1)


def test_too_few_tracklets_are_copied():
    P, w = _frame(19, 200)
    m = O.match(P, w, threads=0)
    idx = m["idx"].copy()
    idx[:3, ::2] = -1           # every other track keeps at most 3
    m2 = dict(m, idx=idx)
    r = _refit(P, m2, w)
    few = (idx >= 0).sum(axis=0) < 4
    assert np.all((r["status"][few] & 64) != 0)
    assert np.array_equal(r["p"][:, few], m["p"][:, few])
    assert np.all(r["n_used"][few] == 0)


def test_indices_that_name_no_tracklet_of_the_layer_are_absent():
    """An index out of range, one whose chamber field is beyond the 540 slots,
    or one naming another layer's tracklet is not that layer's tracklet: the
    refit equals the one with -1 there."""
    P, w = _frame(23, 200)
    m = O.match(P, w, threads=0)
    w2 = dict(w)
    dr = w["tkl_det_row"].copy()
    ntk = dr.size
    bogus = ntk
    dr = np.concatenate([dr, np.array([(600 << 5) | 3, ((2 ** 27 - 1) << 5) | 1], np.uint32)])
    w2["tkl_det_row"] = dr
    for k in ("tkl_y", "tkl_z", "tkl_dy"):
        w2[k] = np.concatenate([w[k], [1.0, 2.0]])
    idx = m["idx"].copy()
    clean = idx.copy()
    idx[0, 0::5] = bogus            # chamber 600: none
    idx[1, 1::5] = bogus + 1        # chamber 2^27 - 1: none
    idx[2, 2::5] = 10 ** 7          # out of range
    idx[3, 3::5] = idx[4, 3::5]     # layer 4's tracklet given for layer 3
    for l, s in ((0, 0), (1, 1), (2, 2), (3, 3)):
        clean[l, s::5] = -1
    r = O.refit(P, dict(p=m["p"], x=m["x"], sector=m["sector"]), idx, w2)
    c = O.refit(P, dict(p=m["p"], x=m["x"], sector=m["sector"]), clean, w2)
    for k in ("p", "cov", "x", "sector", "chi2", "n_used", "status"):
        assert np.array_equal(r[k], c[k]), k
    assert (c["n_used"] < m["n_match"]).sum() > 50
