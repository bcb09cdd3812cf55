"""Pins of the oracle's decision-margin flags: each flag fires for a decision
that lies inside its margin and stays silent just outside it.

Every case is one track in a group of its own, in a geometry whose road is a
closed form: no field (straight tracks), no material, no tilt, seed at
x = 250 cm with sin(phi) = 0 and a diagonal covariance.  At the first layer
(dx = 40 cm) the innovation covariance is then S_yy = C_yy + dx^2 C_ss +
sigma_y^2, S_zz = C_zz + dx^2 C_tt + pad^2/12, S_yz = 0, the road half widths
are n_road sqrt(S), and the dy gate is n_dy sqrt(sigma_dy^2 + L^2 C_ss).  The
candidates are placed at chosen fractions of those limits (computed here,
not by the oracle), and the flags of the first layer are compared with the
rule of each flag:
  P1  the winner within the margin of one of its gates;
  P2  a candidate that fails exactly one gate within the margin and would
      otherwise have won;
  P3  a runner-up chi2 within the margin of the winner's;
  P4  the sector edge, the z acceptance of the search window, or snp_max
      within the margin;
and, with P1 and P2, which gate the decision concerned: the chi2 cut (the
class the parity contract names) or a road edge / the dy gate.
Margin: 1e-4 relative to the limit plus the absolute term of the precision
(none for double; the float terms are checked on their own cases).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2003_03174_amd import synth

P1, P2, P3, P4 = O.FL_P1, O.FL_P2, O.FL_P3, O.FL_P4
CUT, GATE = O.FL_KCUT, O.FL_KGATE
X0, DX = 250.0, 40.0
CYY, CZZ, CSS, CTT = 0.01, 0.04, 1e-6, 1e-6
Z0 = 4.0      # a pad-row centre
IN, OUT = 0.5e-4, 3e-4    # fractions inside and outside the 1e-4 margin


def _params(**over):
    P = synth.default_params(bz=0.0, x_over_x0=0.0, **over)
    return P


def _road(P):
    """Closed-form innovation covariance, road and dy gate at the first layer."""
    vy = P["sigma_y"][0] ** 2
    syy = CYY + DX * DX * CSS + vy
    szz = CZZ + DX * DX * CTT + P["pad_len"] ** 2 / 12.0
    gdy = P["n_sigma_dy"] * math.sqrt(P["sigma_dy"][0] ** 2 + P["drift_len"] ** 2 * CSS)
    return syy, szz, P["n_sigma_road"] * math.sqrt(syy), P["n_sigma_road"] * math.sqrt(szz), gdy


class Case:
    """One track (own group) with its first-layer candidates (ry, rz, ddy)
    relative to the prediction, and the expected flags and match."""

    def __init__(self, name, cands, flags, match, y0=0.0, z0=Z0, s0=0.0, kind=0):
        self.name, self.cands, self.flags, self.match = name, cands, flags, match
        self.kind = kind if flags & (P1 | P2) else 0   # CUT / GATE: the gate of a P1 or P2 decision
        self.y0, self.z0, self.s0 = y0, z0, s0


def _workload(P, cases):
    n = len(cases)
    p = np.zeros((5, n))
    cov = np.zeros((15, n))
    for i, c in enumerate(cases):
        p[:, i] = (c.y0, c.z0, c.s0, 0.0, 1.0)
    for k, v in zip((0, 5, 9, 12, 14), (CYY, CZZ, CSS, CTT, 1e-4)):
        cov[k] = v
    ys, zs, dys, drs, gs = [], [], [], [], []
    tan10 = math.tan(math.pi / 18)
    for i, c in enumerate(cases):
        f = math.sqrt(1.0 - c.s0 * c.s0)
        yl = c.y0 + DX * c.s0 / f            # straight line to the first layer
        dytrk = P["drift_len"] * (c.s0 / f - P["tan_psi"])
        sec = 0 if abs(yl) <= P["x_layer"][0] * tan10 else (1 if yl > 0 else 17)
        for ry, rz, ddy in c.cands:
            z = c.z0 + rz
            row = int(math.floor((z - P["z_min"]) / P["pad_len"]))
            det = sec * 30 + (row // P["n_rows"]) * 6 + 0
            ys.append(yl + ry)
            zs.append(z)
            dys.append(dytrk + ddy)
            drs.append((det << 5) | (row % P["n_rows"]))
            gs.append(i)
    return dict(p=p, cov=cov, x=np.full(n, X0), sector=np.zeros(n, np.int32),
                group=np.arange(n, dtype=np.int32), n_groups=n,
                tkl_y=np.array(ys), tkl_z=np.array(zs), tkl_dy=np.array(dys),
                tkl_det_row=np.array(drs, dtype=np.uint32), tkl_group=np.array(gs, dtype=np.int32))


def _check(P, cases, margins):
    w = _workload(P, cases)
    for mode in ("binned", "brute"):
        o = O.match(P, w, mode=mode, threads=2, margins=margins)
        for i, c in enumerate(cases):
            got = int(o["flags"][i])
            assert got & O.FL_DECISIONS == c.flags, (mode, c.name, got, c.flags)
            assert got & (CUT | GATE) == c.kind, (mode, c.name, got, c.kind)
            if c.flags:
                assert o["flag_layer"][i] == 0, (mode, c.name)
            assert (o["idx"][0, i] >= 0) == c.match, (mode, c.name)


def test_chi2_cut_margin_double():
    P = _params()
    c2max = P["chi2_max"]
    syy, szz, _, _, _ = _road(P)
    cases = []
    for d, flag_pass, flag_fail in ((IN, P1, P2), (OUT, 0, 0)):
        rz = math.sqrt(szz)          # chi2 contribution 1, far inside the z road
        ry_in = math.sqrt(syy * (c2max * (1 - d) - 1.0))
        ry_out = math.sqrt(syy * (c2max * (1 + d) - 1.0))
        cases.append(Case(f"pass {d}", [(ry_in, rz, 0.0)], flag_pass, True, kind=CUT))
        cases.append(Case(f"fail {d}", [(-ry_out, -rz, 0.0)], flag_fail, False, kind=CUT))
    _check(P, cases, dict(margin_rel=1e-4))


def test_road_edge_margin_double():
    """n_road = 3: the road box lies inside the chi2 ellipse's box, so the
    road edges are the deciding gates."""
    P = _params(n_sigma_road=3.0)
    _, _, ry_lim, rz_lim, _ = _road(P)
    cases = []
    for d, fp, ff in ((IN, P1, P2), (OUT, 0, 0)):
        cases.append(Case(f"y pass {d}", [(ry_lim * (1 - d), 0.0, 0.0)], fp, True, kind=GATE))
        cases.append(Case(f"y fail {d}", [(-ry_lim * (1 + d), 0.0, 0.0)], ff, False, kind=GATE))
        cases.append(Case(f"z pass {d}", [(0.0, rz_lim * (1 - d), 0.0)], fp, True, kind=GATE))
        cases.append(Case(f"z fail {d}", [(0.0, -rz_lim * (1 + d), 0.0)], ff, False, kind=GATE))
    _check(P, cases, dict(margin_rel=1e-4))


def test_dy_gate_margin_double():
    P = _params()
    _, _, _, _, gdy = _road(P)
    cases = []
    for d, fp, ff in ((IN, P1, P2), (OUT, 0, 0)):
        cases.append(Case(f"pass {d}", [(0.0, 0.0, gdy * (1 - d))], fp, True, kind=GATE))
        cases.append(Case(f"fail {d}", [(0.0, 0.0, -gdy * (1 + d))], ff, False, kind=GATE))
    _check(P, cases, dict(margin_rel=1e-4))


def test_p2_needs_a_loser_that_would_win():
    """A loser failing the dy gate by a margin flags the track only if its
    chi2 is at most the winner's (within the margin)."""
    P = _params()
    syy, _, _, _, gdy = _road(P)
    win = (math.sqrt(2.0 * syy), 0.0, 0.0)                    # chi2 = 2
    cases = [
        Case("better loser", [win, (math.sqrt(1.0 * syy), 0.0, gdy * (1 + IN))], P2, True, kind=GATE),
        Case("worse loser", [win, (-math.sqrt(3.0 * syy), 0.0, gdy * (1 + IN))], 0, True),
        Case("better loser far", [win, (math.sqrt(1.0 * syy), 0.0, gdy * (1 + OUT))], 0, True),
        # a loser failing two gates, one of them by a margin, never flags
        Case("two gates", [win, (math.sqrt(13.8155 * 1.2 * syy), 0.0, gdy * (1 + IN))], 0, True),
    ]
    _check(P, cases, dict(margin_rel=1e-4))


def test_p2_needs_exactly_one_failed_gate():
    """n_road = 3.  A loser with a smaller chi2 than the winner that fails the
    z road (by 7 %) and the dy gate (within the margin) fails two gates: no
    flag.  The same loser inside the z road fails one: P2."""
    P = _params(n_sigma_road=3.0)
    syy, szz, _, _, gdy = _road(P)
    win = (2.9 * math.sqrt(syy), 2.2 * math.sqrt(szz), 0.0)          # chi2 = 13.25
    cases = [
        Case("two gates", [win, (0.0, -3.2 * math.sqrt(szz), gdy * (1 + IN))], 0, True),
        Case("one gate", [win, (0.0, -2.9 * math.sqrt(szz), gdy * (1 + IN))], P2, True, kind=GATE),
    ]
    _check(P, cases, dict(margin_rel=1e-4))


def test_near_tie_margin_double():
    P = _params()
    syy, _, _, _, _ = _road(P)
    cases = []
    for d, f in ((IN, P3), (OUT, 0)):
        cases.append(Case(f"tie {d}", [(math.sqrt(2.0 * syy), 0.0, 0.0),
                                       (-math.sqrt(2.0 * (1 + d) * syy), 0.0, 0.0)], f, True))
    _check(P, cases, dict(margin_rel=1e-4))


def test_sector_edge_z_acceptance_and_snp_margins_double():
    P = _params()
    _, szz, _, rz_lim, _ = _road(P)
    ylim = P["x_layer"][0] * math.tan(math.pi / 18)
    zmax = -P["z_min"]
    cases = []
    for d, f in ((IN, P4), (OUT, 0)):
        cases.append(Case(f"edge in {d}", [], f, False, y0=ylim * (1 - d)))
        cases.append(Case(f"edge out {d}", [], f, False, y0=-ylim * (1 + d)))
        # lower edge of the search window at the upper end of the chambers
        cases.append(Case(f"z {d}", [], f, False, z0=zmax * (1 - d) + rz_lim))
        cases.append(Case(f"z below {d}", [], f, False, z0=zmax * (1 + d) + rz_lim))
        # |sin phi| at snp_max (a steep straight track; y chosen to stay in sector 0)
        s0 = P["snp_max"] * (1 - d)
        cases.append(Case(f"snp {d}", [], f, False, y0=-90.0, s0=s0))
    _check(P, cases, dict(margin_rel=1e-4))


def test_float_margins_add_their_absolute_terms():
    """With the float path's margins (absolute terms from its state
    tolerance: 1e-3 cm on lengths, 2e-4 cm on dy, 2e-2 on chi2) a decision
    within rel * |limit| + abs fires, one at 1.5 times that distance not."""
    m = dict(margin_rel=1e-4, m_len=1e-3, m_dy=2e-4, m_chi2=2e-2, m_snp=1e-5)
    P = _params(n_sigma_road=3.0)
    syy, szz, ry_lim, rz_lim, gdy = _road(P)
    c2max = P["chi2_max"]
    cases = []
    for frac, fp in ((0.6, P1), (1.5, 0)):
        e_y = frac * (1e-4 * ry_lim + 1e-3)
        e_dy = frac * (1e-4 * gdy + 2e-4)
        e_c2 = frac * (1e-4 * c2max + 2e-2)
        cases.append(Case(f"y {frac}", [(ry_lim - e_y, 0.0, 0.0)], fp, True, kind=GATE))
        cases.append(Case(f"dy {frac}", [(0.0, 0.0, gdy - e_dy)], fp, True, kind=GATE))
        # chi2 edge inside the 3 sigma road: rz = 2.5 sigma, ry (2.75 sigma) fills the rest
        ry = math.sqrt(syy * (c2max - e_c2 - 6.25))
        cases.append(Case(f"chi2 {frac}", [(ry, 2.5 * math.sqrt(szz), 0.0)], fp, True, kind=CUT))
    _check(P, cases, m)


def test_state_tolerance_margin_scales_with_the_road():
    """The chi2 margins carry the compared path's state tolerance through
    each road: with y, z errors up to m_state * max(|y|, 10 cm) (here, at
    y = 0, z = 4 cm, no tilt or misalignment: 10 m_state each) a chi2 moves
    by at most kchi sqrt(chi2) + kchi^2 / 4 with kchi = 2 |e| /
    sqrt(lambda_min(S)) = 2 sqrt(2) 10 m_state / sqrt(min(S_yy, S_zz)) for
    this diagonal S.  A near tie or a chi2-cut decision within that (plus
    1e-4 relative) fires, one at 1.5 times the distance not."""
    ms = 1e-4     # large enough that the road term dominates the relative one
    m = dict(margin_rel=1e-4, m_state=ms)
    P = _params(n_sigma_road=6.0)
    syy, szz, _, _, _ = _road(P)
    c2max = P["chi2_max"]
    kchi = 2.0 * math.sqrt(2.0) * 10.0 * ms / math.sqrt(min(syy, szz))

    def err(c2):
        return kchi * math.sqrt(c2) + 0.25 * kchi * kchi

    assert err(c2max) > 20 * 1e-4 * c2max
    cases = []
    for frac, fp in ((0.6, True), (1.5, False)):
        # near tie: winner at chi2 2, runner-up above it by frac of the margin
        c_w = 2.0
        d = frac * (1e-4 * c_w + err(c_w) + err(c_w + 0.2))
        cases.append(Case(f"tie {frac}", [(math.sqrt(c_w * syy), 0.0, 0.0),
                                          (-math.sqrt((c_w + d) * syy), 0.0, 0.0)], P3 if fp else 0, True))
        # chi2 cut: a lone winner just inside the cut
        e_c2 = frac * (1e-4 * c2max + err(c2max))
        ry = math.sqrt(syy * (c2max - e_c2 - 1.0))
        cases.append(Case(f"cut {frac}", [(ry, math.sqrt(szz), 0.0)], P1 if fp else 0, True, kind=CUT))
    _check(P, cases, m)
    # without the state tolerance the same decisions lie outside the margin
    quiet = [Case(c.name, c.cands, 0, True) for c in cases]
    _check(P, quiet, dict(margin_rel=1e-4))
