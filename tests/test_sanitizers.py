"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code,
run on the CPU.

- The FP64 oracle (plain C) built with -fsanitize=address,undefined runs the
  binned, brute-force and several-hypotheses matchers, the binning, the
  TRD-only refit and the residual maps of small workloads (with tilt,
  misalignment, the detector model and invalid inputs).
- The host side of libtrd (the C ABI: argument and config checks, context
  set-up) is built with the sanitizers on the host compilation only and
  driven through every call's argument checks; without a GPU every path that
  needs a device stops at its first HIP call.
Any sanitizer report fails the test (UBSan does not recover).
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN_ENV = dict(ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:exitcode=86",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1:exitcode=87")

ORACLE_SCRIPT = r"""
import numpy as np
from oracle import oracle as O
from paper_2003_03174_amd import synth
P = dict(tilt=synth.tilt_pm2deg(), dx_chamber=np.random.default_rng(1).uniform(-0.5, 0.5, 540))
w = synth.generate(n_tracks=300, seed=5, fake_ratio=0.5, ineff_frac=0.1, params=P)
w["p"] = w["p"].copy(); w["p"][0, 0] = np.nan; w["sector"] = w["sector"].copy(); w["sector"][1] = 40
w["tkl_det_row"] = w["tkl_det_row"].copy(); w["tkl_det_row"][3] = (600 << 5) | 1
for mode in ("binned", "brute"):
    m = O.match(w["params"], w, mode=mode, threads=2, layers=True, margins=dict(margin_rel=1e-4, m_state=1e-5))
perm, off = O.bin_tracklets(w["params"], w)
Q = dict(w["params"], n_hyp=4, chi2_penalty=9.0)
O.match(Q, w, threads=2)
r = O.refit(w["params"], m, m["idx"], w)
cl = synth.tpc_clusters(w, 2)
O.residual_sums(w["params"], r, cl)
wr = synth.generate(n_tracks=200, seed=6, params=synth.realistic_overrides())
O.match(wr["params"], wr, threads=2)
print("oracle-sanitized-ok")
"""

HOST_SCRIPT = r"""
import ctypes as C
from paper_2003_03174_amd import binding as B
from paper_2003_03174_amd import synth
L = B.lib()
for code in (0, -1, -2, -3, -4, -5, 7):
    L.trd_status_string(code)
h = C.c_void_p()
assert L.trd_create(None, 0, C.byref(h)) == B.TRD_EINVAL
c = B.make_config(synth.default_params(), "fp32")
c.n_rows = 99
assert L.trd_create(C.byref(c), 0, C.byref(h)) == B.TRD_EINVAL
c = B.make_config(synth.default_params(), "fp32")
c.y_bin_w = 3.0
assert L.trd_create(C.byref(c), 0, C.byref(h)) == B.TRD_EINVAL
c = B.make_config(synth.default_params(), "fp32")
c.flags = B.TRD_CFG_FAIL_ALLOC
assert L.trd_create(C.byref(c), 0, C.byref(h)) == B.TRD_ENOMEM
c = B.make_config(synth.default_params(), "fp32")
rc = L.trd_create(C.byref(c), 0, C.byref(h))   # no device here: a clean failure
assert rc in (B.TRD_EDEVICE, B.TRD_OK), rc
if rc == B.TRD_OK:
    L.trd_destroy(h)
t = B.trd_tracklets()
assert L.trd_load_tracklets(None, C.byref(t), 0, 1, None) == B.TRD_EINVAL
assert L.trd_match(None, C.byref(B.trd_tracks()), 0, C.byref(B.trd_results()), None) == B.TRD_EINVAL
assert L.trd_match_noalloc(None, C.byref(B.trd_tracks()), 0, C.byref(B.trd_results()), None) == B.TRD_EINVAL
assert L.trd_reserve(None, 1, 1, 1) == B.TRD_EINVAL
assert L.trd_device_bytes(None) == 0
L.trd_destroy(None)
print("host-sanitized-ok")
"""


def _run(script, env_extra, tmp_path):
    env = dict(os.environ, **SAN_ENV, **env_extra)
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    return subprocess.run([sys.executable, "-c", script], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)


def _clean(r, marker):
    bad = ("AddressSanitizer" in r.stderr or "runtime error" in r.stderr or
           "UndefinedBehaviorSanitizer" in r.stderr)
    assert r.returncode == 0 and marker in r.stdout and not bad, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    lib = str(tmp_path / "libtrd_oracle_san.so")
    subprocess.run(["gcc", "-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fPIC", "-shared",
                    "-o", lib, os.path.join(ROOT, "oracle", "trd_oracle.c"), "-lm"], check=True)
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    ubsan = subprocess.run(["gcc", "-print-file-name=libubsan.so"], capture_output=True, text=True).stdout.strip()
    r = _run(ORACLE_SCRIPT, dict(TRD_ORACLE_LIB=lib, LD_PRELOAD=f"{asan} {ubsan}"), tmp_path)
    _clean(r, "oracle-sanitized-ok")


def test_host_abi_under_address_and_undefined_sanitizers(tmp_path):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not found")
    from paper_2003_03174_amd import build as hb
    lib = str(tmp_path / "libtrd_san.so")
    flags = [f for f in hb.HIPCC_FLAGS if not f.startswith("-O")] + [
        "-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
        "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    subprocess.run([hipcc, *flags, "-o", lib] + [os.path.join(hb.CSRC, s) for s in hb.SOURCES], check=True,
                   capture_output=True)
    rt = subprocess.run([hipcc, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True).stdout.strip()
    if not os.path.exists(rt):
        import glob
        found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not found:
            pytest.skip("clang ASan runtime not found")
        rt = found[0]
    r = _run(HOST_SCRIPT, dict(TRD_LIB=lib, LD_PRELOAD=rt), tmp_path)
    _clean(r, "host-sanitized-ok")
