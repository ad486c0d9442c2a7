"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The FP64 oracle, built with gcc's sanitizers, runs gradient, matvec, PCG
  (InvA, InvH0, 2LInvH0), a Gauss-Newton iteration, the transport VJP and the
  standalone operators on four small grids (tests/sanitize/oracle_driver.c);
  leaks are checked too.
* The library's host code (validation, workspace sizing, error paths), built
  with the sanitizers on its host side only (the gfx950 device code is
  compiled as usual), is driven by tests/sanitize/lib_driver.c through the C
  ABI; without a GPU every device-touching call must fail cleanly.
Builds go to tests/sanitize/_build (reused while the sources are unchanged)."""
import hashlib
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
BUILD = os.path.join(SAN, "_build")
CSRC = os.path.join(ROOT, "paper_2008_12820_amd", "csrc")
LIB_SOURCES = ["api.hip", "fft.hip", "transport.hip", "linalg.hip", "batch.hip"]
CLANG = "/opt/rocm/llvm/bin/clang"


def _digest(paths, extra):
    h = hashlib.sha256(extra.encode())
    for p in paths:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    exe = os.path.join(BUILD, "oracle_driver")
    src = [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "lddmm_oracle.c")]
    _run(["gcc", "-std=gnu11", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-fno-omit-frame-pointer", "-fopenmp", *src, "-lm", "-o", exe])
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe], env=env, timeout=300)
    assert "oracle sanitizer run: ok" in r.stdout


@pytest.mark.skipif(shutil.which("hipcc") is None or not os.path.exists(CLANG), reason="needs hipcc and clang")
def test_library_host_code_under_asan_ubsan():
    os.makedirs(BUILD, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-g", "-std=c++20", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-ffp-contract=fast", "-I" + os.path.join(ROOT, "include"), *san]
    srcs = [os.path.join(CSRC, s) for s in LIB_SOURCES]
    headers = [os.path.join(CSRC, h) for h in ("internal.hpp", "common.hpp")] + [
        os.path.join(ROOT, "include", "lddmm.h")]
    key = _digest(srcs + headers, " ".join(flags))
    lib = os.path.join(BUILD, f"liblddmm_san_{key}.so")
    if not os.path.exists(lib):
        procs, objs = [], []
        for s in srcs:
            o = os.path.join(BUILD, os.path.basename(s) + f".{key}.o")
            objs.append(o)
            procs.append(subprocess.Popen(["hipcc", "-c", *flags, s, "-o", o], stdout=subprocess.PIPE,
                                          stderr=subprocess.PIPE, text=True))
        for p in procs:
            _, err = p.communicate()
            assert p.returncode == 0, err[-4000:]
        _run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", *objs, "-o", lib + ".tmp"])
        os.replace(lib + ".tmp", lib)
        for o in objs:
            os.remove(o)
    exe = os.path.join(BUILD, f"lib_driver_{key}")
    _run([CLANG, "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          os.path.join(SAN, "lib_driver.c"), lib, f"-Wl,-rpath,{BUILD}", "-o", exe])
    # the HIP runtime keeps process-lifetime allocations: no leak report
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = _run([exe], env=env, timeout=300)
    assert "library host sanitizer run: ok" in r.stdout, r.stdout
