"""Host-side sanitizer builds (CPU only; no GPU work):
- the CPU oracle's C code under AddressSanitizer and
  UndefinedBehaviorSanitizer (gcc), driven over every entry point on a small
  closed scene;
- the library's host code (argument checks, the tuning-table parser) built
  by hipcc with the sanitizers on the host side only, driven by a host
  program whose every call returns before any device work.
A sanitizer report makes the program exit non-zero."""
import glob
import hashlib
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.returncode, r.stdout[-2000:], r.stderr[-4000:])


def test_oracle_under_asan_ubsan():
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, "oracle_asan")
    subprocess.check_call(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-fno-omit-frame-pointer", "-fopenmp", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off",
                           os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
                           os.path.join(ROOT, "oracle", "uvc_oracle.c"), "-lm", "-o", exe])
    _run(exe)


def test_library_host_paths_under_asan_ubsan():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/lib/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("ROCm compilers not available")
    os.makedirs(OUT, exist_ok=True)
    srcs = sorted(glob.glob(os.path.join(ROOT, "paper_2103_14137_amd", "csrc", "*.hip")) +
                  glob.glob(os.path.join(ROOT, "paper_2103_14137_amd", "csrc", "*.cpp")))
    hdrs = sorted(glob.glob(os.path.join(ROOT, "paper_2103_14137_amd", "csrc", "*.hpp")) +
                  [os.path.join(ROOT, "include", "uvc.h")])
    h = hashlib.sha1()
    for f in srcs + hdrs:
        h.update(open(f, "rb").read())
    lib = os.path.join(OUT, f"libuvc_asan_{h.hexdigest()[:12]}.so")
    if not os.path.exists(lib):
        for old in glob.glob(os.path.join(OUT, "libuvc_asan_*.so")):
            os.remove(old)
        san = []
        for flag in ("-fsanitize=address", "-fsanitize=undefined", "-fno-omit-frame-pointer"):
            san += ["-Xarch_host", flag]  # host code only; the device code is built as usual
        subprocess.check_call([hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared", *san,
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                               "-I" + os.path.join(ROOT, "include"), *srcs, "-o", lib],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    exe = os.path.join(OUT, "abi_asan")
    subprocess.check_call([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                           "-I" + os.path.join(ROOT, "include"),
                           os.path.join(ROOT, "tests", "sanitize", "abi_driver.cpp"), lib, "-Wl,-rpath," + OUT,
                           "-o", exe])
    _run(exe)
