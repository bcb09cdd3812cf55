"""The C-ABI library without a GPU: it loads, exports every symbol the header
declares, and rejects bad arguments before touching a device."""
import ctypes as C
import os
import re

import pytest

from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "trd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(trd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_function():
    L = B.lib()
    declared = _header_functions()
    assert set(declared) == set(B.EXPORTS), declared
    for name in declared:
        assert hasattr(L, name), name


def test_config_struct_size_matches_header_layout():
    # 2 ints + 12 doubles + 2 doubles + 4 ints + 3 doubles + 540 + 3 + 3+3+1 + 4 doubles + u64 + 2 ints
    # + n_hyp (int, padded) + chi2_penalty + refit_cov[5] + refit_min (int, padded)
    # + tpc_x_in, tpc_x_out + 5 ints (padded) + 3 doubles (energy loss) + 540 bytes (padded to 544)
    # + 3 doubles (field map)
    assert C.sizeof(B.trd_config) == (8 + 8 * 12 + 16 + 16 + 24 + 8 * 540 + 24 + 56 + 32 + 8 + 8 + 16 + 48 + 40
                                      + 24 + 544 + 24)


def test_status_strings():
    assert B.trd_status_string(0) == "ok"
    assert B.trd_status_string(-1) == "invalid argument"
    assert B.trd_status_string(-5) == "HBM budget exceeded"
    assert B.trd_status_string(7) == "unknown status"


def _cfg(**kw):
    P = synth.default_params()
    return B.make_config(P, "fp32", **kw)


@pytest.mark.parametrize("mutate", [
    lambda c: setattr(c, "struct_size", 12),
    lambda c: setattr(c, "precision", 7),
    lambda c: setattr(c, "y_bin_w", 3.0),          # not a power of two
    lambda c: setattr(c, "dy_bin_w", 0.1),
    lambda c: setattr(c, "n_db", 0),
    lambda c: setattr(c, "n_rows", 40),
    lambda c: setattr(c, "snp_max", 1.5),
    lambda c: setattr(c, "pad_len", 7.0),          # rows no longer tile [z_min, -z_min]
    lambda c: setattr(c, "block_size", 100),
    lambda c: setattr(c, "block_size", 512),
    lambda c: setattr(c, "search_lanes", 3),
    lambda c: (setattr(c, "search_lanes", 8), setattr(c, "flags", B.TRD_CFG_PERSISTENT)),
    lambda c: setattr(c, "n_hyp", 3),
    lambda c: (setattr(c, "n_hyp", 4), setattr(c, "search_lanes", 8)),
    lambda c: (setattr(c, "n_hyp", 2), setattr(c, "chi2_penalty", -1.0)),
    lambda c: c.refit_cov.__setitem__(3, 0.0),
    lambda c: setattr(c, "refit_min", 0),
    lambda c: setattr(c, "refit_min", 7),
    lambda c: setattr(c, "tpc_n_rows", 1),
    lambda c: setattr(c, "tpc_x_out", 50.0),
    lambda c: setattr(c, "vox_nx", 16),          # 18 * 16 * 4 * 3 > 2048 voxels
    lambda c: setattr(c, "vox_min", 0),
    lambda c: c.x_layer.__setitem__(2, float("nan")),
    lambda c: setattr(c, "eloss_xrho", -1.0),
    lambda c: (setattr(c, "eloss_xrho", 1.0), setattr(c, "eloss_za", 0.0)),
    lambda c: (setattr(c, "eloss_xrho", 1.0), setattr(c, "eloss_i", float("nan"))),
    lambda c: (setattr(c, "eloss_xrho", 1.0), setattr(c, "mass", 0.0)),
])
def test_create_rejects_bad_config(mutate):
    c = _cfg()
    mutate(c)
    h = C.c_void_p()
    assert B.lib().trd_create(C.byref(c), 0, C.byref(h)) == B.TRD_EINVAL
    assert not h.value


def test_injected_allocation_failure():
    c = _cfg(flags=B.TRD_CFG_FAIL_ALLOC)
    h = C.c_void_p()
    assert B.lib().trd_create(C.byref(c), 0, C.byref(h)) == B.TRD_ENOMEM


def test_null_context_calls():
    L = B.lib()
    t = B.trd_tracklets()
    assert L.trd_load_tracklets(None, C.byref(t), 0, 1, None) == B.TRD_EINVAL
    assert L.trd_match(None, C.byref(B.trd_tracks()), 0, C.byref(B.trd_results()), None) == B.TRD_EINVAL
    assert L.trd_match_noalloc(None, C.byref(B.trd_tracks()), 0, C.byref(B.trd_results()), None) == B.TRD_EINVAL
    assert L.trd_load_and_match(None, C.byref(t), 0, 1, C.byref(B.trd_tracks()), 0, C.byref(B.trd_results()),
                                None) == B.TRD_EINVAL
    assert L.trd_reserve(None, 1, 1, 1) == B.TRD_EINVAL
    assert L.trd_device_bytes(None) == 0
    L.trd_destroy(None)


def test_product_path_has_no_cpu_fallback():
    """The binding refuses to run without a device instead of computing on the CPU."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        B.Matcher(synth.default_params(), "fp32")
