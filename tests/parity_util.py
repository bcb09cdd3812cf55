"""Element-by-element comparison of the HIP path's results with the FP64 oracle.

Norms (relative errors with floors): y, z: 10 cm; sin phi, tan lambda: 0.1;
q/pT: 0.1 c/GeV; covariance entries: |dC_ij| / sqrt(C_ii C_jj).

Tolerances:
  * double path: 1e-12 on state and covariance;
  * float path: 1e-5 on the state; the float covariance is reported (its
    Joseph-form update is bounded by positive definiteness, not by 1e-5) and
    checked against a loose bound;
  * chi2: the state tolerance carried through the residual,
    |d chi2| <= 6 layers * 2 sqrt(chi2_max) / sigma_y * (tol * 10 cm).
Index parity: a track whose oracle run holds a decision-margin flag is
compared (indices and chi2 per layer) only on the layers before the first
flagged layer (there, a different but correct rounding may legitimately pick
another candidate); its final state is not compared.  The report counts the
flagged tracks per flag, and separately those whose only flagged decisions
concern the chi2 cut (the near-cut class of the contract); every test bounds
the flagged share (`max_flag_share`).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

FLOORS = np.array([10.0, 10.0, 0.1, 0.1, 0.1])
DIAG = (0, 5, 9, 12, 14)
GPU_ONLY_BITS = 8 | 16   # FP64_FALLBACK, NOT_PD
FL_P1, FL_P2, FL_P3, FL_P4, FL_KCUT, FL_KGATE = 1, 2, 4, 8, 16, 32

# ceilings on the share of flagged (exempt) tracks: a planted mistake that
# over-flags would otherwise leave every parity test green.  Double: the
# 1e-4 relative margin alone; float: plus the absolute terms below.
MAX_FLAG_SHARE = {"fp64": 0.01, "fp32": 0.06, "fp32_cov64": 0.06}
# several hypotheses: every comparison of path costs at every layer can flag
# (frames of up to 20k tracks; the wide roads of displaced seeds hold many
# near-equal paths)
MAX_FLAG_SHARE_BEAM = 0.15
MAX_FLAG_SHARE_BEAM_WIDE = 0.25

STATE_TOL = {"fp64": 1e-12, "fp32": 1e-5, "fp32_cov64": 1e-5}
COV_TOL = {"fp64": 1e-12, "fp32": 5e-2, "fp32_cov64": 5e-2}

# decision margins the oracle uses to flag tracks for each precision (the
# absolute terms follow from the state tolerance: 1e-5 * 10 cm on y and z)
# (m_ke: a track left with less than this fraction of its kinetic energy by a
# layer's loss has a momentum whose relative error is the precision's times
# the inverse fraction: 1e-3 keeps double within 1e-12, 0.02 float within 1e-5)
# (m_state: the state tolerance, carried through each road's innovation
# covariance into the chi2 comparisons; it replaces a fixed absolute chi2 term
# derived from the narrowest road)
MARGINS = {
    "fp64": dict(margin_rel=1e-4, m_ke=1e-3, m_state=1e-12),
    "fp32": dict(margin_rel=1e-4, m_len=1e-3, m_dy=2e-4, m_snp=1e-5, m_ke=2e-2, m_state=1e-5),
    "fp32_cov64": dict(margin_rel=1e-4, m_len=1e-3, m_dy=2e-4, m_snp=1e-5, m_ke=2e-2, m_state=1e-5),
}
# Several hypotheses compare sums of chi2 over the layers: there the float
# margin keeps a fixed absolute term of 2e-2 (the state tolerance 1e-4 cm
# carried through the narrowest road, 2 sqrt(chi2_max) / sigma_y per layer's
# residual pair) in place of the per-road term.
BEAM_MARGINS = {k: dict(v, m_chi2=(0.0 if k == "fp64" else 2e-2)) for k, v in MARGINS.items()}


def tilted_float_tol(P, y_max=None):
    """State bound of the float paths with tilted pads.  The y measurement
    of a tilted pad row depends on z, so the update turns a y residual error
    into a z error with the gain K_zy = tau C_zz / S_yy, largest for a track
    whose z is known to a pad row, C_zz = pad^2 / 12: with tan 2 deg, 8 cm
    rows and sigma_y = 0.04 cm, K_zy ~ 23.  The float state holds y (up to
    the sector half width at the outer layer, 65 cm) to a unit roundoff u =
    2^-24 at best, so z takes an extra u y_max K_zy: relative to the 10 cm
    floor, 1e-5 + u * 65 * 23 / 10 ~ 1.9e-5."""
    tau = max(abs(t) for t in P["tilt"])
    czz = P["pad_len"] ** 2 / 12.0
    s = np.linspace(-P["snp_max"], P["snp_max"], 2001)
    sy = float(np.min(np.abs(np.polyval(list(P["sigma_y"])[::-1], s))))   # narrowest width
    k_zy = tau * czz / (tau * tau * czz + sy * sy)
    if y_max is None:
        y_max = max(P["x_layer"]) * math.tan(math.pi / 18) + 0.5
    return STATE_TOL["fp32"] + 2.0 ** -24 * y_max * k_zy / FLOORS[1]


def chi2_tol(prec, chi2_max=13.8155, sigma_y=0.04):
    return 6 * 2 * math.sqrt(chi2_max) / sigma_y * STATE_TOL[prec] * 10.0


@dataclass
class Report:
    prec: str
    n: int = 0
    n_flagged: int = 0
    n_compared: int = 0
    idx_mismatch: int = 0
    idx_mismatch_flagged_prefix: int = 0
    status_mismatch: int = 0
    sector_mismatch: int = 0
    nmatch_mismatch: int = 0
    state_err: float = 0.0
    state_err_q999: float = 0.0
    state_tol: float = 0.0
    q999_tol: float = 0.0
    state_err_by_comp: list = field(default_factory=list)
    x_err: float = 0.0
    cov_err: float = 0.0
    chi2_err: float = 0.0
    n_fallback: int = 0
    chi2_layer_err: float = 0.0
    chi2_layer_mismatch_flagged_prefix: int = 0
    flag_counts: dict = field(default_factory=dict)
    n_flag_cut_only: int = 0
    max_flag_share: float = 0.0
    bad_tracks: list = field(default_factory=list)

    @property
    def flag_share(self):
        return self.n_flagged / self.n if self.n else 0.0

    @property
    def ok(self):
        tol = self.state_tol or STATE_TOL[self.prec]
        return (self.idx_mismatch == 0 and self.idx_mismatch_flagged_prefix == 0 and
                self.status_mismatch == 0 and self.sector_mismatch == 0 and
                self.nmatch_mismatch == 0 and self.state_err <= tol and
                self.state_err_q999 <= (self.q999_tol or STATE_TOL[self.prec]) and
                self.x_err <= STATE_TOL[self.prec] and self.cov_err <= COV_TOL[self.prec] and
                self.chi2_err <= chi2_tol(self.prec) and self.chi2_layer_err <= chi2_tol(self.prec) and
                self.chi2_layer_mismatch_flagged_prefix == 0 and
                self.flag_share <= (self.max_flag_share or MAX_FLAG_SHARE[self.prec]))

    def summary(self):
        fc = " ".join(f"{k}={v}" for k, v in self.flag_counts.items())
        return (f"{self.prec}: n={self.n} flagged={self.n_flagged} ({fc} cut_only={self.n_flag_cut_only}) "
                f"compared={self.n_compared} "
                f"idx_mm={self.idx_mismatch}+{self.idx_mismatch_flagged_prefix} "
                f"status_mm={self.status_mismatch} sec_mm={self.sector_mismatch} "
                f"nm_mm={self.nmatch_mismatch} state={self.state_err:.3g} q999={self.state_err_q999:.3g} "
                f"by_comp={[f'{v:.2g}' for v in self.state_err_by_comp]} x={self.x_err:.3g} "
                f"cov={self.cov_err:.3g} chi2={self.chi2_err:.3g} chi2_layer={self.chi2_layer_err:.3g}"
                f"+{self.chi2_layer_mismatch_flagged_prefix} fallback={self.n_fallback} "
                f"ok={self.ok}")


def compare(ref, got, prec, sel=None, state_tol_max=None, q999_tol=None, max_flag_share=None):
    """ref: oracle.match output; got: numpy copies of the device results
    (same keys).  sel: optional index array of tracks that `ref` covers
    (ref holds len(sel) tracks, got holds all).  state_tol_max: a looser
    bound on the worst track; q999_tol: a looser bound on the 99.9 %
    quantile of the per-track error (default: the state tolerance);
    max_flag_share: ceiling on the flagged share (default MAX_FLAG_SHARE)."""
    g = dict(got)
    if sel is not None:
        sel = np.asarray(sel)
        for k in ("idx", "p", "cov", "chi2_layer"):
            if g.get(k) is not None:
                g[k] = g[k][:, sel]
        for k in ("x", "sector", "chi2", "n_match", "status"):
            g[k] = g[k][sel]
    n = ref["x"].size
    r = Report(prec=prec, n=n, state_tol=state_tol_max or 0.0, q999_tol=q999_tol or 0.0,
               max_flag_share=max_flag_share or 0.0)
    fbits = ref["flags"].astype(np.int64)
    flagged = fbits != 0
    fl = ref["flag_layer"]
    r.n_flagged = int(flagged.sum())
    r.flag_counts = {nm: int(((fbits & b) != 0).sum()) for nm, b in
                     (("P1", FL_P1), ("P2", FL_P2), ("P3", FL_P3), ("P4", FL_P4))}
    r.n_flag_cut_only = int((flagged & ((fbits & (FL_P3 | FL_P4 | FL_KGATE)) == 0) &
                             ((fbits & FL_KCUT) != 0)).sum())
    gst = g["status"].astype(np.int64)
    r.n_fallback = int(((gst & 8) != 0).sum())
    # indices: all layers of unflagged tracks, the layers before the flag otherwise
    layer = np.arange(6)[:, None]
    cmp_mask = layer < fl[None, :]
    mm = (g["idx"] != ref["idx"]) & cmp_mask
    r.idx_mismatch = int(mm[:, ~flagged].any(axis=0).sum())
    r.idx_mismatch_flagged_prefix = int(mm[:, flagged].any(axis=0).sum())
    # chi2 per layer where both matched the same tracklet on a compared layer
    if g.get("chi2_layer") is not None:
        tol = chi2_tol(prec)
        both = cmp_mask & (g["idx"] == ref["idx"]) & (ref["idx"] >= 0)
        d = np.abs(g["chi2_layer"].astype(np.float64) - ref["chi2_layer"])
        d = np.where(both, d, 0.0)
        if d[:, ~flagged].size:
            r.chi2_layer_err = float(d[:, ~flagged].max())
        if d[:, flagged].size:
            r.chi2_layer_mismatch_flagged_prefix = int((d[:, flagged] > tol).any(axis=0).sum())
    u = ~flagged
    r.n_compared = int(u.sum())
    st_g = (gst & ~GPU_ONLY_BITS)[u]
    r.status_mismatch = int((st_g != ref["status"][u].astype(np.int64)).sum())
    r.sector_mismatch = int((g["sector"][u] != ref["sector"][u]).sum())
    r.nmatch_mismatch = int((g["n_match"][u] != ref["n_match"][u]).sum())
    # rejected seeds are copied through (NaN included) on both sides
    bad_in = (ref["status"] & 32) != 0
    for k in ("p", "cov"):
        if not np.array_equal(g[k][:, bad_in].astype(np.float64), ref[k][:, bad_in], equal_nan=True):
            r.status_mismatch += 1
    same = u & ~bad_in & (g["sector"] == ref["sector"]) & ((gst & ~GPU_ONLY_BITS) == ref["status"])
    same &= np.all(g["idx"] == ref["idx"], axis=0)
    if same.any():
        gp, rp = g["p"][:, same].astype(np.float64), ref["p"][:, same]
        e = np.abs(gp - rp) / np.maximum(np.abs(rp), FLOORS[:, None])
        r.state_err_by_comp = [float(v) for v in e.max(axis=1)]
        r.state_err = float(e.max())
        r.state_err_q999 = float(np.quantile(e.max(axis=0), 0.999))
        r.x_err = float((np.abs(g["x"][same].astype(np.float64) - ref["x"][same]) /
                         np.maximum(np.abs(ref["x"][same]), 1.0)).max())
        gc, rc = g["cov"][:, same].astype(np.float64), ref["cov"][:, same]
        k = 0
        worst = 0.0
        for i in range(5):
            for j in range(i, 5):
                den = np.sqrt(rc[DIAG[i]] * rc[DIAG[j]])
                worst = max(worst, float((np.abs(gc[k] - rc[k]) / den).max()))
                k += 1
        r.cov_err = worst
        r.chi2_err = float(np.abs(g["chi2"][same].astype(np.float64) - ref["chi2"][same]).max())
        if r.state_err > STATE_TOL[prec]:
            bad = np.nonzero(same)[0][np.argsort(-e.max(axis=0))[:5]]
            r.bad_tracks = [int(b) for b in bad]
    return r


def to_numpy(out):
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}
