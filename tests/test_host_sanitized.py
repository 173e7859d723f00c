"""Host code under the sanitizers (no GPU needed).

* ``tests/host/host_logic_probe.cpp``: the series time index, the serving
  arena (first fit, coalescing), the admission rule (arrival order, no
  overtaking) and the tick planner (block budget, fair share, every row
  launched once) from ``csrc/rr_host.h``, the code the library runs, checked
  against brute-force models with AddressSanitizer and
  UndefinedBehaviorSanitizer (built with g++).
* ``tests/host/asan_abi_calls.py``: a build of librr.so whose host code
  carries AddressSanitizer (the device code is unchanged), loaded in a
  child process with the ASan runtime preloaded and Python allocating
  through malloc (so every argument buffer has redzones); it runs the
  C-ABI's host-side validation -- rr_prepare_ld over grids and profiles,
  rr_series_create's checks and index construction over hundreds of series,
  every entry point's NULL paths -- and fails on any memory error or
  unexpected return code.  A planted one-past-the-end read of the pbids
  array in rr_series_create was reported by this run as a heap-buffer-overflow.
"""

import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2009_08500_amd", "csrc")
SOURCES = ["rr_capi.hip", "rr_prep.hip", "rr_forward.hip", "rr_adjoint.hip", "rr_serve.hip"]


def _tool(name, *cands):
    for c in (*cands, shutil.which(name)):
        if c and os.path.exists(c):
            return c
    pytest.skip(f"{name} not available")


def test_host_logic_under_asan_and_ubsan(tmp_path):
    gxx = _tool("g++")
    exe = str(tmp_path / "host_logic_probe")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-I", CSRC,
                    os.path.join(ROOT, "tests", "host", "host_logic_probe.cpp"), "-o", exe],
                   check=True, capture_output=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK")
    assert "runtime error" not in r.stderr


def _asan_runtime():
    clang = _tool("clang", "/opt/rocm/llvm/bin/clang")
    path = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                          capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("ASan runtime not found")
    return path


def test_c_abi_host_validation_under_asan(tmp_path):
    hipcc = _tool("hipcc", os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc")
    runtime = _asan_runtime()
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-fvisibility=hidden",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-fno-omit-frame-pointer",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs, procs = [], []
    for s in SOURCES:
        o = str(tmp_path / s.replace(".hip", ".o"))
        objs.append(o)
        procs.append(subprocess.Popen([hipcc, *flags, "-c", os.path.join(CSRC, s), "-o", o],
                                      stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True))
    for p in procs:
        _, err = p.communicate(timeout=600)
        assert p.returncode == 0, err
    lib = str(tmp_path / "librr_asan.so")
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host",
                    "-fsanitize=address", "-shared-libasan", *objs, "-o", lib],
                   check=True, capture_output=True)
    env = dict(os.environ, LD_PRELOAD=runtime, PYTHONMALLOC="malloc",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host", "asan_abi_calls.py"),
                        lib, os.path.join(ROOT, "paper_2009_08500_amd", "_lib.py")],
                       capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out, out
    assert r.returncode == 0, out
    assert r.stdout.strip().endswith("OK"), out
