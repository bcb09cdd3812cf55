"""ctypes front end of the FP64 CPU oracle (trd_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg
of the benchmark import this module; the product path never does.  It takes
the plain parameter dict of a workload and numpy arrays, and shares no code
with the HIP library or its binding.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "trd_oracle.c")
_LIB = os.environ.get("TRD_ORACLE_LIB") or os.path.join(_HERE, "libtrd_oracle.so")

ST_STOP_SNP, ST_ROT_FAIL, ST_OUT_OF_Z, ST_BAD_INPUT = 1, 2, 4, 32
ST_STOPPED = 256
FL_P1, FL_P2, FL_P3, FL_P4 = 1, 2, 4, 8
FL_KCUT, FL_KGATE = 16, 32   # the gate a P1/P2 decision concerned: the chi2 cut, a road edge or the dy gate
FL_DECISIONS = FL_P1 | FL_P2 | FL_P3 | FL_P4


class OCfg(C.Structure):
    _fields_ = [
        ("x_layer", C.c_double * 6),
        ("tilt", C.c_double * 6),
        ("z_min", C.c_double), ("pad_len", C.c_double),
        ("y_bin_w", C.c_double), ("dy_bin_w", C.c_double), ("drift_len", C.c_double),
        ("dx_chamber", C.c_double * 540),
        ("bz", C.c_double), ("x_over_x0", C.c_double), ("mass", C.c_double),
        ("sigma_y", C.c_double * 3), ("sigma_dy", C.c_double * 3), ("tan_psi", C.c_double),
        ("chi2_max", C.c_double), ("n_sigma_dy", C.c_double), ("n_sigma_road", C.c_double),
        ("snp_max", C.c_double),
        ("m_rel", C.c_double), ("m_len", C.c_double), ("m_dy", C.c_double),
        ("m_chi2", C.c_double), ("m_snp", C.c_double),
        ("n_rows", C.c_int32), ("n_yb", C.c_int32), ("n_db", C.c_int32),
        ("n_hyp", C.c_int32), ("chi2_penalty", C.c_double),
        ("refit_cov", C.c_double * 5), ("refit_min", C.c_int32), ("pad_", C.c_int32),
        ("eloss_xrho", C.c_double), ("eloss_za", C.c_double), ("eloss_i", C.c_double),
        ("absent", C.c_uint8 * 540), ("pad2_", C.c_uint8 * 4), ("m_ke", C.c_double),
        ("m_state", C.c_double),
        ("field_br", C.c_double), ("field_bz", C.c_double), ("field_step", C.c_double),
    ]

class OTpc(C.Structure):
    _fields_ = [("x_in", C.c_double), ("x_out", C.c_double), ("n_rows", C.c_int32),
                ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("min_count", C.c_int32),
                ("pad_", C.c_int32)]


# sub-volumes of the residual maps: per sector 8 in x, 4 in y/x, 3 in z/x
VOXELS = (8, 4, 3)
VOXEL_MIN = 20


# TRD-only refit defaults: starting covariance diag (cm^2, cm^2, -, -, (c/GeV)^2)
REFIT_COV = (1.0, 100.0, 1e-2, 1e-2, 1.0)
REFIT_MIN = 4


def build(force=False):
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP).  A library
    named by TRD_ORACLE_LIB (a planted-mistake variant in a check of the
    pins) is used as it is."""
    if os.environ.get("TRD_ORACLE_LIB"):
        return _LIB
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-std=gnu11", "-O2", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-unused-function", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_LIB)
        dp, ip, up, lp = (C.POINTER(C.c_double), C.POINTER(C.c_int32),
                          C.POINTER(C.c_uint32), C.POINTER(C.c_int64))
        L.oracle_cfg_size.restype = C.c_int32
        L.oracle_bin.argtypes = [C.POINTER(OCfg), C.c_int64, dp, dp, dp, up, ip, C.c_int32, ip, up]
        L.oracle_match.argtypes = ([C.POINTER(OCfg), C.c_int64, dp, dp, dp, ip, ip,
                                    C.c_int64, dp, dp, dp, up, ip, C.c_int32, C.c_int32, C.c_int32,
                                    ip, dp, dp, dp, ip, dp, dp, ip, up, up, ip, lp, dp, dp, dp, ip, dp])
        L.oracle_refit.argtypes = [C.POINTER(OCfg), C.c_int64, dp, dp, ip, ip, C.c_int64, dp, dp, up,
                                   C.c_int32, dp, dp, dp, ip, dp, ip, up]
        L.oracle_residuals.argtypes = [C.POINTER(OCfg), C.POINTER(OTpc), C.c_int64, dp, dp, ip, up, lp, dp, dp,
                                       ip, ip, dp]
        L.oracle_voxel_solve.argtypes = [C.POINTER(OTpc), C.c_int64, dp, dp]
        L.oracle_propagate.argtypes = [C.POINTER(OCfg), dp, dp, dp, C.c_double, dp]
        L.oracle_rotate.argtypes = [C.POINTER(OCfg), dp, dp, dp, C.c_double, dp]
        L.oracle_add_ms.argtypes = [C.POINTER(OCfg), dp, dp]
        L.oracle_eloss.argtypes = [C.POINTER(OCfg), dp, dp, C.c_int]
        L.oracle_bethe.argtypes = [C.POINTER(OCfg), C.c_double, C.c_double]
        L.oracle_bethe.restype = C.c_double
        L.oracle_chamber_at.argtypes = [C.POINTER(OCfg), C.c_int, C.c_int, C.c_double]
        L.oracle_update.argtypes = [dp, dp, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double]
        L.oracle_ldl_pd.argtypes = [dp]
        L.oracle_key.argtypes = [C.POINTER(OCfg), C.c_double, C.c_double, C.c_double, C.c_uint32,
                                 C.c_int32, C.c_int32]
        L.oracle_key.restype = C.c_int64
        assert L.oracle_cfg_size() == C.sizeof(OCfg), "oracle config layout mismatch"
        _lib = L
    return _lib


def make_cfg(params, margin_rel=1e-4, m_len=0.0, m_dy=0.0, m_chi2=0.0, m_snp=0.0, m_ke=1e-3, m_state=0.0):
    c = OCfg()
    P = params
    for l in range(6):
        c.x_layer[l] = P["x_layer"][l]
        c.tilt[l] = P["tilt"][l]
    c.z_min, c.pad_len = P["z_min"], P["pad_len"]
    c.y_bin_w, c.drift_len = P["y_bin_w"], P["drift_len"]
    c.dy_bin_w, c.n_db = P["dy_bin_w"], P["n_db"]
    for d in range(540):
        c.dx_chamber[d] = float(P["dx_chamber"][d])
    c.bz, c.x_over_x0, c.mass = P["bz"], P["x_over_x0"], P["mass"]
    for k in range(3):
        c.sigma_y[k] = P["sigma_y"][k]
        c.sigma_dy[k] = P["sigma_dy"][k]
    c.tan_psi = P["tan_psi"]
    c.chi2_max, c.n_sigma_dy = P["chi2_max"], P["n_sigma_dy"]
    c.n_sigma_road, c.snp_max = P["n_sigma_road"], P["snp_max"]
    c.m_rel, c.m_len, c.m_dy, c.m_chi2, c.m_snp = margin_rel, m_len, m_dy, m_chi2, m_snp
    c.m_ke = m_ke
    c.m_state = m_state
    c.field_br = float(P.get("field_br", 0.0))
    c.field_bz = float(P.get("field_bz", 0.0))
    c.field_step = float(P.get("field_step", 0.25))
    c.n_rows, c.n_yb = P["n_rows"], P["n_yb"]
    c.n_hyp = int(P.get("n_hyp", 0))
    c.chi2_penalty = float(P.get("chi2_penalty", P["chi2_max"]))
    for k in range(5):
        c.refit_cov[k] = float(P.get("refit_cov", REFIT_COV)[k])
    c.refit_min = int(P.get("refit_min", REFIT_MIN))
    c.eloss_xrho = float(P.get("eloss_xrho", 0.0))
    c.eloss_za = float(P.get("eloss_za", 0.5))
    c.eloss_i = float(P.get("eloss_i", 1e-7))
    ab = P.get("absent")
    if ab is not None:
        ab = np.asarray(ab).reshape(540)
        for d in range(540):
            c.absent[d] = 1 if ab[d] else 0
    return c


def _ptr(a, t):
    return a.ctypes.data_as(C.POINTER(t)) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def bin_tracklets(params, w):
    """Sorted permutation and cell offsets of the workload's tracklets."""
    L = lib()
    cfg = make_cfg(params)
    n = int(w["tkl_y"].size)
    ng = int(w.get("n_groups", 1))
    nc = ng * 540 * params["n_rows"] * params["n_db"] * params["n_yb"]
    y, z, dy = _f64(w["tkl_y"]), _f64(w["tkl_z"]), _f64(w["tkl_dy"])
    dr = np.ascontiguousarray(w["tkl_det_row"], dtype=np.uint32)
    g = np.ascontiguousarray(w["tkl_group"], dtype=np.int32) if "tkl_group" in w else None
    perm = np.zeros(max(n, 1), np.int32)
    off = np.zeros(nc + 1, np.uint32)
    rc = L.oracle_bin(C.byref(cfg), n, _ptr(y, C.c_double), _ptr(z, C.c_double), _ptr(dy, C.c_double),
                      _ptr(dr, C.c_uint32), _ptr(g, C.c_int32), ng, _ptr(perm, C.c_int32),
                      _ptr(off, C.c_uint32))
    assert rc == 0
    return perm[:n], off


def match(params, w, *, mode="binned", threads=0, layers=False, margins=None, track_slice=None):
    """Run the oracle on a workload dict (see synth.generate).

    margins: dict(margin_rel, m_len, m_dy, m_chi2, m_snp) for the decision
    flags.  track_slice: optional index array of tracks to process (the rest
    of the workload's tracklets stay in the search).
    Returns a dict of numpy outputs.
    """
    L = lib()
    cfg = make_cfg(params, **(margins or {}))
    tp, tc, tx = _f64(w["p"]), _f64(w["cov"]), _f64(w["x"])
    ts = np.ascontiguousarray(w["sector"], dtype=np.int32)
    tg = np.ascontiguousarray(w["group"], dtype=np.int32) if "group" in w else None
    if track_slice is not None:
        sl = np.asarray(track_slice)
        tp, tc, tx, ts = (np.ascontiguousarray(tp[:, sl]), np.ascontiguousarray(tc[:, sl]),
                          np.ascontiguousarray(tx[sl]), np.ascontiguousarray(ts[sl]))
        tg = np.ascontiguousarray(tg[sl]) if tg is not None else None
    n = int(tx.size)
    y, z, dy = _f64(w["tkl_y"]), _f64(w["tkl_z"]), _f64(w["tkl_dy"])
    dr = np.ascontiguousarray(w["tkl_det_row"], dtype=np.uint32)
    kg = np.ascontiguousarray(w["tkl_group"], dtype=np.int32) if "tkl_group" in w else None
    ng = int(w.get("n_groups", 1))
    o = dict(
        idx=np.zeros((6, n), np.int32), p=np.zeros((5, n)), cov=np.zeros((15, n)),
        x=np.zeros(n), sector=np.zeros(n, np.int32), chi2=np.zeros(n),
        chi2_layer=np.zeros((6, n)), n_match=np.zeros(n, np.int32),
        status=np.zeros(n, np.uint32), flags=np.zeros(n, np.uint32),
        flag_layer=np.zeros(n, np.int32), n_cand=np.zeros(n, np.int64), cost=np.zeros(n),
    )
    if layers:
        o.update(lp=np.zeros((6, 5, n)), lc=np.zeros((6, 15, n)), lx=np.zeros((6, n)),
                 lsec=np.zeros((6, n), np.int32))
    dp, ip, up = C.c_double, C.c_int32, C.c_uint32
    rc = L.oracle_match(
        C.byref(cfg), n, _ptr(tp, dp), _ptr(tc, dp), _ptr(tx, dp), _ptr(ts, ip), _ptr(tg, ip),
        int(y.size), _ptr(y, dp), _ptr(z, dp), _ptr(dy, dp), _ptr(dr, up), _ptr(kg, ip), ng,
        1 if mode == "brute" else 0, int(threads),
        _ptr(o["idx"], ip), _ptr(o["p"], dp), _ptr(o["cov"], dp), _ptr(o["x"], dp),
        _ptr(o["sector"], ip), _ptr(o["chi2"], dp), _ptr(o["chi2_layer"], dp),
        _ptr(o["n_match"], ip), _ptr(o["status"], up), _ptr(o["flags"], up),
        _ptr(o["flag_layer"], ip), _ptr(o["n_cand"], C.c_int64),
        _ptr(o.get("lp"), dp), _ptr(o.get("lc"), dp), _ptr(o.get("lx"), dp), _ptr(o.get("lsec"), ip),
        _ptr(o["cost"], dp))
    assert rc == 0, rc
    return o


def refit(params, tracks, idx, w, threads=0):
    """TRD-only refit of matched tracks.  tracks: dict with p [5][n], x, sector
    (e.g. the output of match()); idx [6][n] the matched tracklet indices;
    w: the workload's tracklets.  Returns p, cov, x, sector, chi2, n_used, status."""
    L = lib()
    cfg = make_cfg(params)
    tp, tx = _f64(tracks["p"]), _f64(tracks["x"])
    ts = np.ascontiguousarray(tracks["sector"], dtype=np.int32)
    ix = np.ascontiguousarray(idx, dtype=np.int32)
    n = int(tx.size)
    y, z = _f64(w["tkl_y"]), _f64(w["tkl_z"])
    dr = np.ascontiguousarray(w["tkl_det_row"], dtype=np.uint32)
    o = dict(p=np.zeros((5, n)), cov=np.zeros((15, n)), x=np.zeros(n), sector=np.zeros(n, np.int32),
             chi2=np.zeros(n), n_used=np.zeros(n, np.int32), status=np.zeros(n, np.uint32))
    dp, ip_, up = C.c_double, C.c_int32, C.c_uint32
    rc = L.oracle_refit(C.byref(cfg), n, _ptr(tp, dp), _ptr(tx, dp), _ptr(ts, ip_), _ptr(ix, ip_),
                        int(y.size), _ptr(y, dp), _ptr(z, dp), _ptr(dr, up), int(threads),
                        _ptr(o["p"], dp), _ptr(o["cov"], dp), _ptr(o["x"], dp), _ptr(o["sector"], ip_),
                        _ptr(o["chi2"], dp), _ptr(o["n_used"], ip_), _ptr(o["status"], up))
    assert rc == 0, rc
    return o


def make_tpc(tpc, voxels=VOXELS, min_count=VOXEL_MIN):
    t = OTpc()
    t.x_in, t.x_out, t.n_rows = float(tpc["x_in"]), float(tpc["x_out"]), int(tpc["n_rows"])
    t.nx, t.ny, t.nz = (int(v) for v in voxels)
    t.min_count = int(min_count)
    return t


def residual_sums(params, ref, cl, voxels=VOXELS):
    """Per-voxel sums [n_vox, 8] of the clusters' residuals against the
    reference tracks (ref: p [5][n], x, sector, status), cl: tpc_clusters()."""
    L = lib()
    cfg = make_cfg(params)
    t = make_tpc(cl["tpc"], voxels)
    n = int(np.asarray(ref["x"]).size)
    nvox = 18 * int(np.prod(voxels))
    sums = np.zeros((nvox, 8))
    rp, rx = _f64(ref["p"]), _f64(ref["x"])
    rs = np.ascontiguousarray(ref["sector"], dtype=np.int32)
    st = np.ascontiguousarray(ref["status"], dtype=np.uint32)
    first = np.ascontiguousarray(cl["first"], dtype=np.int64)
    cy, cz = _f64(cl["y"]), _f64(cl["z"])
    crow = np.ascontiguousarray(cl["row"], dtype=np.int32)
    csec = np.ascontiguousarray(cl["sector"], dtype=np.int32)
    dp, ip_, up, lp = C.c_double, C.c_int32, C.c_uint32, C.c_int64
    rc = L.oracle_residuals(C.byref(cfg), C.byref(t), n, _ptr(rp, dp), _ptr(rx, dp), _ptr(rs, ip_), _ptr(st, up),
                            _ptr(first, lp), _ptr(cy, dp), _ptr(cz, dp), _ptr(crow, ip_), _ptr(csec, ip_),
                            _ptr(sums, dp))
    assert rc == 0
    return sums


def voxel_solve(sums, tpc, voxels=VOXELS, min_count=VOXEL_MIN):
    """(dX, dY, dZ, n) per voxel from residual_sums()."""
    t = make_tpc(tpc, voxels, min_count)
    s = np.ascontiguousarray(sums, dtype=np.float64)
    out = np.zeros((s.shape[0], 4))
    lib().oracle_voxel_solve(C.byref(t), s.shape[0], _ptr(s, C.c_double), _ptr(out, C.c_double))
    return out


# ---- single steps -----------------------------------------------------------

def _cfg_only(params):
    return make_cfg(params)


def propagate(params, p, cov, x, x2, want_j=False):
    """One helix step.  Returns (ok, p, cov, x, J)."""
    L = lib()
    cfg = _cfg_only(params)
    p = _f64(p).copy()
    cv = _f64(cov).copy() if cov is not None else None
    xx = np.array([x], dtype=np.float64)
    J = np.zeros(25)
    ok = L.oracle_propagate(C.byref(cfg), _ptr(p, C.c_double), _ptr(cv, C.c_double),
                            _ptr(xx, C.c_double), float(x2), _ptr(J, C.c_double))
    return bool(ok), p, cv, float(xx[0]), J.reshape(5, 5)


def rotate(params, p, cov, x, da):
    L = lib()
    cfg = _cfg_only(params)
    p = _f64(p).copy()
    cv = _f64(cov).copy() if cov is not None else None
    xx = np.array([x], dtype=np.float64)
    J = np.zeros(25)
    ok = L.oracle_rotate(C.byref(cfg), _ptr(p, C.c_double), _ptr(cv, C.c_double),
                         _ptr(xx, C.c_double), float(da), _ptr(J, C.c_double))
    return bool(ok), p, cv, float(xx[0]), J.reshape(5, 5)


def add_ms(params, p, cov):
    L = lib()
    cfg = _cfg_only(params)
    p = _f64(p).copy()
    cv = _f64(cov).copy()
    L.oracle_add_ms(C.byref(cfg), _ptr(p, C.c_double), _ptr(cv, C.c_double))
    return cv


def eloss(params, p, cov, direction=1):
    """The layer's mean energy loss at the state p (direction +1 outward,
    -1 inward).  Returns (ok, p, cov)."""
    L = lib()
    cfg = _cfg_only(params)
    p = _f64(p).copy()
    cv = _f64(cov).copy()
    ok = L.oracle_eloss(C.byref(cfg), _ptr(p, C.c_double), _ptr(cv, C.c_double), int(direction))
    return bool(ok), p, cv


def bethe(params, p, m):
    """Mean energy loss rate (GeV cm^2/g) of the oracle's material model."""
    return float(lib().oracle_bethe(C.byref(_cfg_only(params)), float(p), float(m)))


def chamber_at(params, sec, layer, z):
    return int(lib().oracle_chamber_at(C.byref(_cfg_only(params)), int(sec), int(layer), float(z)))


def update(p, cov, ry, rz, tau, vy, vz):
    L = lib()
    p = _f64(p).copy()
    cv = _f64(cov).copy()
    L.oracle_update(_ptr(p, C.c_double), _ptr(cv, C.c_double), ry, rz, tau, vy, vz)
    return p, cv


def ldl_pd(cov):
    return bool(lib().oracle_ldl_pd(_ptr(_f64(cov).copy(), C.c_double)))


def key(params, y, z, dy, det_row, grp=0, n_groups=1):
    cfg = _cfg_only(params)
    return int(lib().oracle_key(C.byref(cfg), y, z, dy, det_row, grp, n_groups))


def unpack(pk):
    """Packed upper-triangular 15-vector -> symmetric 5x5 (numpy, for tests)."""
    M = np.zeros((5, 5))
    k = 0
    for i in range(5):
        for j in range(i, 5):
            M[i, j] = M[j, i] = pk[k]
            k += 1
    return M


def pack(M):
    return np.array([M[i, j] for i in range(5) for j in range(i, 5)])
