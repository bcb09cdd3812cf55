"""Python binding of libtrd (include/trd.h): argument marshalling only.

Every step of the matching runs in the HIP kernels of libtrd.so; this module
packs plain parameters into `trd_config`, hands torch device tensors to the C
ABI as raw pointers and raises on error codes.  Torch provides device memory
and streams, nothing else.  There is no CPU fallback: without the built
library (or a GPU) every call fails loudly.
"""
from __future__ import annotations

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TRD_LIB: another build of the same library (a sanitizer build in a CPU test)
LIB_PATH = os.environ.get("TRD_LIB") or os.path.join(HERE, "libtrd.so")

TRD_OK, TRD_EINVAL, TRD_ENOMEM, TRD_EDEVICE, TRD_ESTATE, TRD_EBUDGET = 0, -1, -2, -3, -4, -5
TRD_PREC_FP64, TRD_PREC_FP32, TRD_PREC_FP32_COV64 = 0, 1, 2
PRECISIONS = {"fp64": TRD_PREC_FP64, "fp32": TRD_PREC_FP32, "fp32_cov64": TRD_PREC_FP32_COV64}
TRK_STOP_SNP, TRK_ROT_FAIL, TRK_OUT_OF_Z, TRK_FP64_FALLBACK, TRK_NOT_PD, TRK_BAD_INPUT = 1, 2, 4, 8, 16, 32
TRK_REFIT_FEW, TRK_REFIT_SKIP, TRK_STOPPED = 64, 128, 256
# TRD-only refit defaults: starting covariance diag (cm^2, cm^2, -, -, (c/GeV)^2), fewest tracklets
REFIT_COV = (1.0, 100.0, 1e-2, 1e-2, 1.0)
REFIT_MIN = 4
# residual maps: TPC pad rows and voxels per sector (x, y/x, z/x), fewest clusters per voxel
TPC_ROWS = dict(x_in=85.0, x_out=245.0, n_rows=64)
VOXELS = (8, 4, 3)
VOXEL_MIN = 20
TRD_CFG_FAIL_ALLOC = 1
TRD_CFG_FORCE_FALLBACK = 2
TRD_CFG_PERSISTENT = 4
TRD_CFG_INPUT_ORDER = 8
TRD_CFG_TIME_KERNEL = 16

# every symbol include/trd.h declares
EXPORTS = ("trd_create", "trd_reserve", "trd_load_tracklets", "trd_match", "trd_match_noalloc",
           "trd_load_and_match", "trd_refit",
           "trd_residual_sums",
           "trd_voxel_solve", "trd_get_binning", "trd_copy_binning", "trd_device_bytes", "trd_kernel_times",
           "trd_destroy", "trd_status_string")


class TrdError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {trd_status_string(code)} ({code})")
        self.code = code


class trd_config(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("precision", C.c_int32),
        ("x_layer", C.c_double * 6), ("tilt", C.c_double * 6),
        ("z_min", C.c_double), ("pad_len", C.c_double),
        ("n_rows", C.c_int32), ("n_yb", C.c_int32), ("n_db", C.c_int32), ("flags", C.c_uint32),
        ("y_bin_w", C.c_double), ("dy_bin_w", C.c_double), ("drift_len", C.c_double),
        ("dx_chamber", C.c_double * 540),
        ("bz", C.c_double), ("x_over_x0", C.c_double), ("mass", C.c_double),
        ("sigma_y", C.c_double * 3), ("sigma_dy", C.c_double * 3), ("tan_psi", C.c_double),
        ("chi2_max", C.c_double), ("n_sigma_dy", C.c_double), ("n_sigma_road", C.c_double),
        ("snp_max", C.c_double),
        ("hbm_budget_bytes", C.c_uint64), ("block_size", C.c_int32), ("search_lanes", C.c_int32),
        ("n_hyp", C.c_int32), ("chi2_penalty", C.c_double),
        ("refit_cov", C.c_double * 5), ("refit_min", C.c_int32),
        ("tpc_x_in", C.c_double), ("tpc_x_out", C.c_double), ("tpc_n_rows", C.c_int32),
        ("vox_nx", C.c_int32), ("vox_ny", C.c_int32), ("vox_nz", C.c_int32), ("vox_min", C.c_int32),
        ("eloss_xrho", C.c_double), ("eloss_za", C.c_double), ("eloss_i", C.c_double),
        ("chamber_absent", C.c_uint8 * 540),
        ("field_br", C.c_double), ("field_bz", C.c_double), ("field_step", C.c_double),
    ]


class trd_tracklets(C.Structure):
    _fields_ = [("y", C.c_void_p), ("z", C.c_void_p), ("dy", C.c_void_p),
                ("det_row", C.c_void_p), ("group", C.c_void_p)]


class trd_tracks(C.Structure):
    _fields_ = [("p", C.c_void_p), ("cov", C.c_void_p), ("x", C.c_void_p),
                ("sector", C.c_void_p), ("group", C.c_void_p)]


class trd_results(C.Structure):
    _fields_ = [("idx", C.c_void_p), ("p", C.c_void_p), ("cov", C.c_void_p), ("x", C.c_void_p),
                ("sector", C.c_void_p), ("chi2", C.c_void_p), ("chi2_layer", C.c_void_p),
                ("n_match", C.c_void_p), ("status", C.c_void_p)]


class trd_refit_in(C.Structure):
    _fields_ = [("p", C.c_void_p), ("x", C.c_void_p), ("sector", C.c_void_p), ("idx", C.c_void_p)]


class trd_refit_out(C.Structure):
    _fields_ = [("p", C.c_void_p), ("cov", C.c_void_p), ("x", C.c_void_p), ("sector", C.c_void_p),
                ("chi2", C.c_void_p), ("n_used", C.c_void_p), ("status", C.c_void_p)]


class trd_reference(C.Structure):
    _fields_ = [("p", C.c_void_p), ("x", C.c_void_p), ("sector", C.c_void_p), ("status", C.c_void_p)]


class trd_tpc_clusters(C.Structure):
    _fields_ = [("y", C.c_void_p), ("z", C.c_void_p), ("row_sec", C.c_void_p), ("first", C.c_void_p)]


class trd_binning_view(C.Structure):
    _fields_ = [("offsets", C.c_void_p), ("sorted", C.c_void_p),
                ("n_cells", C.c_int64), ("n_tracklets", C.c_int64)]


_lib = None


def lib():
    """The loaded libtrd.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.trd_create.argtypes = [C.POINTER(trd_config), C.c_int, C.POINTER(vp)]
        L.trd_reserve.argtypes = [vp, C.c_int64, C.c_int32, C.c_int64]
        L.trd_load_tracklets.argtypes = [vp, C.POINTER(trd_tracklets), C.c_int64, C.c_int32, vp]
        L.trd_match.argtypes = [vp, C.POINTER(trd_tracks), C.c_int64, C.POINTER(trd_results), vp]
        L.trd_match_noalloc.argtypes = [vp, C.POINTER(trd_tracks), C.c_int64, C.POINTER(trd_results), vp]
        L.trd_load_and_match.argtypes = [vp, C.POINTER(trd_tracklets), C.c_int64, C.c_int32, C.POINTER(trd_tracks),
                                         C.c_int64, C.POINTER(trd_results), vp]
        L.trd_refit.argtypes = [vp, C.POINTER(trd_refit_in), C.POINTER(trd_tracklets), C.c_int64, C.c_int64,
                                C.POINTER(trd_refit_out), vp]
        L.trd_residual_sums.argtypes = [vp, C.POINTER(trd_reference), C.POINTER(trd_tpc_clusters), C.c_int64,
                                        C.c_int64, vp, vp]
        L.trd_voxel_solve.argtypes = [vp, vp, vp, vp]
        L.trd_get_binning.argtypes = [vp, C.POINTER(trd_binning_view)]
        L.trd_copy_binning.argtypes = [vp, vp, vp, C.c_int64, vp]
        L.trd_device_bytes.argtypes = [vp]
        L.trd_device_bytes.restype = C.c_int64
        L.trd_kernel_times.argtypes = [vp, C.POINTER(C.c_float), C.c_int32]
        L.trd_destroy.argtypes = [vp]
        L.trd_destroy.restype = None
        L.trd_status_string.argtypes = [C.c_int]
        L.trd_status_string.restype = C.c_char_p
        _lib = L
    return _lib


def trd_status_string(code: int) -> str:
    return lib().trd_status_string(int(code)).decode()


def _check(rc, what):
    if rc != TRD_OK:
        raise TrdError(rc, what)


def make_config(params, precision="fp32", *, budget_bytes=0, block_size=0, search_lanes=0, flags=0):
    """trd_config from the plain parameter dict of a workload."""
    c = trd_config()
    c.struct_size = C.sizeof(trd_config)
    c.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    for l in range(6):
        c.x_layer[l] = float(params["x_layer"][l])
        c.tilt[l] = float(params["tilt"][l])
    c.z_min, c.pad_len = float(params["z_min"]), float(params["pad_len"])
    c.n_rows, c.n_yb = int(params["n_rows"]), int(params["n_yb"])
    c.y_bin_w, c.drift_len = float(params["y_bin_w"]), float(params["drift_len"])
    c.n_db, c.dy_bin_w = int(params["n_db"]), float(params["dy_bin_w"])
    for d in range(540):
        c.dx_chamber[d] = float(params["dx_chamber"][d])
    c.bz, c.x_over_x0, c.mass = float(params["bz"]), float(params["x_over_x0"]), float(params["mass"])
    for k in range(3):
        c.sigma_y[k] = float(params["sigma_y"][k])
        c.sigma_dy[k] = float(params["sigma_dy"][k])
    c.tan_psi = float(params["tan_psi"])
    c.chi2_max, c.n_sigma_dy = float(params["chi2_max"]), float(params["n_sigma_dy"])
    c.n_sigma_road, c.snp_max = float(params["n_sigma_road"]), float(params["snp_max"])
    c.hbm_budget_bytes = int(budget_bytes)
    c.block_size = int(block_size)
    c.search_lanes = int(search_lanes)
    c.flags = int(flags)
    c.n_hyp = int(params.get("n_hyp", 0))
    c.chi2_penalty = float(params.get("chi2_penalty", params["chi2_max"]))
    for k in range(5):
        c.refit_cov[k] = float(params.get("refit_cov", REFIT_COV)[k])
    c.refit_min = int(params.get("refit_min", REFIT_MIN))
    tpc = params.get("tpc", TPC_ROWS)
    c.tpc_x_in, c.tpc_x_out, c.tpc_n_rows = float(tpc["x_in"]), float(tpc["x_out"]), int(tpc["n_rows"])
    c.vox_nx, c.vox_ny, c.vox_nz = (int(v) for v in params.get("voxels", VOXELS))
    c.vox_min = int(params.get("vox_min", VOXEL_MIN))
    c.eloss_xrho = float(params.get("eloss_xrho", 0.0))
    c.eloss_za = float(params.get("eloss_za", 0.5))
    c.eloss_i = float(params.get("eloss_i", 1e-7))
    ab = params.get("absent")
    if ab is not None:
        for d, v in enumerate(list(ab)[:540]):
            c.chamber_absent[d] = 1 if v else 0
    c.field_br = float(params.get("field_br", 0.0))
    c.field_bz = float(params.get("field_bz", 0.0))
    c.field_step = float(params.get("field_step", 0.25))
    return c


# ---- C-ABI calls under their own names ------------------------------------

def trd_create(cfg: trd_config, device: int = 0) -> int:
    h = C.c_void_p()
    _check(lib().trd_create(C.byref(cfg), int(device), C.byref(h)), "trd_create")
    return h.value


def trd_reserve(ctx, max_tracklets, max_groups, max_tracks):
    _check(lib().trd_reserve(ctx, int(max_tracklets), int(max_groups), int(max_tracks)), "trd_reserve")


def trd_load_tracklets(ctx, t: trd_tracklets, n, n_groups, stream=0):
    _check(lib().trd_load_tracklets(ctx, C.byref(t), int(n), int(n_groups), stream or None),
           "trd_load_tracklets")


def trd_load_and_match(ctx, t: trd_tracklets, n_tkl, n_groups, trk: trd_tracks, n, res: trd_results, stream=0):
    _check(lib().trd_load_and_match(ctx, C.byref(t), int(n_tkl), int(n_groups), C.byref(trk), int(n),
                                    C.byref(res), stream or None), "trd_load_and_match")


def trd_match(ctx, trk: trd_tracks, n, res: trd_results, stream=0):
    _check(lib().trd_match(ctx, C.byref(trk), int(n), C.byref(res), stream or None), "trd_match")


def trd_match_noalloc(ctx, trk: trd_tracks, n, res: trd_results, stream=0):
    _check(lib().trd_match_noalloc(ctx, C.byref(trk), int(n), C.byref(res), stream or None),
           "trd_match_noalloc")


def trd_refit(ctx, rin: trd_refit_in, tkl: trd_tracklets, n_tkl, n, rout: trd_refit_out, stream=0):
    _check(lib().trd_refit(ctx, C.byref(rin), C.byref(tkl), int(n_tkl), int(n), C.byref(rout), stream or None),
           "trd_refit")


def trd_residual_sums(ctx, ref: trd_reference, cl: trd_tpc_clusters, n, n_cl, sums_ptr, stream=0):
    _check(lib().trd_residual_sums(ctx, C.byref(ref), C.byref(cl), int(n), int(n_cl), sums_ptr, stream or None),
           "trd_residual_sums")


def trd_voxel_solve(ctx, sums_ptr, dist_ptr, stream=0):
    _check(lib().trd_voxel_solve(ctx, sums_ptr, dist_ptr, stream or None), "trd_voxel_solve")


def trd_get_binning(ctx) -> trd_binning_view:
    v = trd_binning_view()
    _check(lib().trd_get_binning(ctx, C.byref(v)), "trd_get_binning")
    return v


def trd_copy_binning(ctx, offsets_ptr, sorted_ptr, max_valid, stream=0):
    _check(lib().trd_copy_binning(ctx, offsets_ptr, sorted_ptr, int(max_valid), stream or None),
           "trd_copy_binning")


def trd_device_bytes(ctx) -> int:
    return int(lib().trd_device_bytes(ctx))


def trd_kernel_times(ctx, max_n=64):
    """Durations (ms) of the main match kernel of the recent trd_match calls."""
    buf = (C.c_float * max(1, max_n))()
    rc = lib().trd_kernel_times(ctx, buf, int(max_n))
    _check(min(rc, 0), "trd_kernel_times")
    return [float(buf[k]) for k in range(rc)]


def trd_destroy(ctx):
    if ctx:
        lib().trd_destroy(ctx)


# ---- torch-facing convenience ------------------------------------------------

def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


class Matcher:
    """One context: tracklets stay resident on the device between matches.

    Tensors passed in must be contiguous device tensors in the layouts of
    include/trd.h (component-major [k][n] for p and cov).
    """

    def __init__(self, params, precision="fp32", device=0, budget_bytes=0, block_size=0,
                 search_lanes=0, flags=0):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("the TRD matcher needs a HIP device")
        self.params = params
        self.precision = precision
        self.device = device
        self.cfg = make_config(params, precision, budget_bytes=budget_bytes, block_size=block_size,
                               search_lanes=search_lanes, flags=flags)
        self.ctx = trd_create(self.cfg, device)
        self.fdtype = torch.float64 if precision == "fp64" else torch.float32
        self.n_tracklets = 0
        self.n_groups = 1

    def close(self):
        if self.ctx:
            trd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reserve(self, max_tracklets, max_groups, max_tracks):
        trd_reserve(self.ctx, max_tracklets, max_groups, max_tracks)

    def load(self, y, z, dy, det_row, group=None, n_groups=1, stream=None):
        self._keep_in = (y, z, dy, det_row, group)
        for t in (y, z, dy, det_row) + ((group,) if group is not None else ()):
            assert t.is_cuda and t.is_contiguous()
        t = trd_tracklets(y.data_ptr(), z.data_ptr(), dy.data_ptr(), det_row.data_ptr(),
                          group.data_ptr() if group is not None else None)
        trd_load_tracklets(self.ctx, t, y.numel(), n_groups, _stream_handle(stream))
        self.n_tracklets = int(y.numel())
        self.n_groups = int(n_groups)

    def alloc_results(self, n, chi2_layer=True):
        import torch
        dev = torch.device("cuda", self.device)
        f = self.fdtype
        return dict(
            idx=torch.empty((6, n), dtype=torch.int32, device=dev),
            p=torch.empty((5, n), dtype=f, device=dev),
            cov=torch.empty((15, n), dtype=f, device=dev),
            x=torch.empty(n, dtype=f, device=dev),
            sector=torch.empty(n, dtype=torch.int32, device=dev),
            chi2=torch.empty(n, dtype=f, device=dev),
            chi2_layer=torch.empty((6, n), dtype=f, device=dev) if chi2_layer else None,
            n_match=torch.empty(n, dtype=torch.int32, device=dev),
            status=torch.empty(n, dtype=torch.int32, device=dev),
        )

    def match(self, p, cov, x, sector, group=None, out=None, stream=None, noalloc=False):
        """trd_match (or trd_match_noalloc with `noalloc`) into `out` (a dict
        of device tensors as alloc_results gives; allocated if None)."""
        n = int(x.numel())
        for t in (p, cov, x):
            assert t.is_cuda and t.is_contiguous() and t.dtype == self.fdtype
        assert sector.is_cuda and sector.is_contiguous()
        if out is None:
            out = self.alloc_results(n)
        trk = trd_tracks(p.data_ptr(), cov.data_ptr(), x.data_ptr(), sector.data_ptr(),
                         group.data_ptr() if group is not None else None)
        res = trd_results(*(None if out[k] is None else out[k].data_ptr() for k in
                            ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status")))
        (trd_match_noalloc if noalloc else trd_match)(self.ctx, trk, n, res, _stream_handle(stream))
        return out

    def load_and_match(self, y, z, dy, det_row, group, n_groups, p, cov, x, sector, tgroup=None, out=None,
                       stream=None):
        """load() then match() in one trd_load_and_match call (the seeds are
        ordered while the tracklets are binned); `group` the tracklets'
        groups, `tgroup` the tracks'."""
        n = int(x.numel())
        for t in (y, z, dy, det_row) + ((group,) if group is not None else ()):
            assert t.is_cuda and t.is_contiguous()
        for t in (p, cov, x):
            assert t.is_cuda and t.is_contiguous() and t.dtype == self.fdtype
        assert sector.is_cuda and sector.is_contiguous()
        self._keep_in = (y, z, dy, det_row, group)
        if out is None:
            out = self.alloc_results(n)
        tk = trd_tracklets(y.data_ptr(), z.data_ptr(), dy.data_ptr(), det_row.data_ptr(),
                           group.data_ptr() if group is not None else None)
        trk = trd_tracks(p.data_ptr(), cov.data_ptr(), x.data_ptr(), sector.data_ptr(),
                         tgroup.data_ptr() if tgroup is not None else None)
        res = trd_results(*(None if out[k] is None else out[k].data_ptr() for k in
                            ("idx", "p", "cov", "x", "sector", "chi2", "chi2_layer", "n_match", "status")))
        trd_load_and_match(self.ctx, tk, y.numel(), n_groups, trk, n, res, _stream_handle(stream))
        self.n_tracklets = int(y.numel())
        self.n_groups = int(n_groups)
        return out

    def refit(self, matched, y, z, det_row, stream=None):
        """TRD-only refit of the tracks of a match() result `matched` (p, x,
        sector, idx) against the tracklets (y, z, det_row) they index."""
        import torch
        n = int(matched["x"].numel())
        dev = torch.device("cuda", self.device)
        f = self.fdtype
        out = dict(p=torch.empty((5, n), dtype=f, device=dev), cov=torch.empty((15, n), dtype=f, device=dev),
                   x=torch.empty(n, dtype=f, device=dev), sector=torch.empty(n, dtype=torch.int32, device=dev),
                   chi2=torch.empty(n, dtype=f, device=dev), n_used=torch.empty(n, dtype=torch.int32, device=dev),
                   status=torch.empty(n, dtype=torch.int32, device=dev))
        rin = trd_refit_in(matched["p"].data_ptr(), matched["x"].data_ptr(), matched["sector"].data_ptr(),
                           matched["idx"].data_ptr())
        tkl = trd_tracklets(y.data_ptr(), z.data_ptr(), None, det_row.data_ptr(), None)
        rout = trd_refit_out(*(out[k].data_ptr() for k in ("p", "cov", "x", "sector", "chi2", "n_used", "status")))
        trd_refit(self.ctx, rin, tkl, y.numel(), n, rout, _stream_handle(stream))
        return out

    def residual_map(self, ref, cl, sums=None, stream=None):
        """Voxel sums [n_vox, 8] (float64, added to `sums` if given) and the
        distortion vectors [n_vox, 4] of the clusters `cl` (device tensors y,
        z float32, row_sec int32, first int64) against the reference tracks
        `ref` (p, x, sector, status; e.g. a refit() result)."""
        import torch
        dev = torch.device("cuda", self.device)
        nx, ny, nz = self.params.get("voxels", VOXELS)
        nv = 18 * int(nx) * int(ny) * int(nz)
        if sums is None:
            sums = torch.zeros((nv, 8), dtype=torch.float64, device=dev)
        n = int(ref["x"].numel())
        r = trd_reference(ref["p"].data_ptr(), ref["x"].data_ptr(), ref["sector"].data_ptr(),
                          ref["status"].data_ptr())
        c = trd_tpc_clusters(cl["y"].data_ptr(), cl["z"].data_ptr(), cl["row_sec"].data_ptr(),
                             cl["first"].data_ptr())
        h = _stream_handle(stream)
        trd_residual_sums(self.ctx, r, c, n, cl["y"].numel(), C.c_void_p(sums.data_ptr()), h)
        dist = torch.empty((nv, 4), dtype=torch.float32, device=dev)
        trd_voxel_solve(self.ctx, C.c_void_p(sums.data_ptr()), C.c_void_p(dist.data_ptr()), h)
        return sums, dist

    def binning(self, stream=None):
        """(offsets[n_cells+1] uint32 as int32, sorted[n_valid, 4] float32) copies."""
        import torch
        v = trd_get_binning(self.ctx)
        dev = torch.device("cuda", self.device)
        off = torch.empty(v.n_cells + 1, dtype=torch.int32, device=dev)
        srt = torch.empty((max(v.n_tracklets, 1), 4), dtype=torch.float32, device=dev)
        trd_copy_binning(self.ctx, off.data_ptr(), srt.data_ptr(), max(v.n_tracklets, 1),
                         _stream_handle(stream))
        return off, srt

    @property
    def device_bytes(self):
        return trd_device_bytes(self.ctx)

    def kernel_times(self, max_n=64):
        """Match-kernel durations of the calls since the last read (needs
        flags=TRD_CFG_TIME_KERNEL)."""
        return trd_kernel_times(self.ctx, max_n)


def device_inputs(dev_layout, precision="fp32", device=0):
    """Device tensors from synth.to_device_layout() arrays."""
    import numpy as np
    import torch
    d = torch.device("cuda", device)
    f = np.float64 if precision == "fp64" else np.float32

    def T(a, dt=None):
        a = np.ascontiguousarray(a if dt is None else a.astype(dt))
        return torch.from_numpy(a).to(d)

    L = dev_layout
    return dict(
        p=T(L["p32"], f), cov=T(L["cov32"], f), x=T(L["x32"], f), sector=T(L["sector"]),
        group=T(L["group"]), y=T(L["y32"]), z=T(L["z32"]), dy=T(L["dy32"]),
        det_row=T(L["det_row"].view(np.int32)), tgroup=T(L["tgroup"]),
    )
