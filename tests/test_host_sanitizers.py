"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host side (the C-ABI argument checks, the hierarchy builder,
the order-independent sums' windows) is compiled with the sanitizers on its
host pass only (each -fsanitize after -Xarch_host; the gfx950 code is built
but never run here) and driven by tests/sanitize/host_checks.cpp; the FP64
oracle's transport is compiled with g++ and the sanitizers and driven by
tests/sanitize/oracle_checks.cpp (every surface kind, gradients, hashes and
recorded branch probabilities). Either run must end cleanly: the sanitizers
abort on their first report."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2604_15017_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SOURCES = ["api", "transport", "image", "replay", "mesh", "splat", "optim"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


def test_oracle_transport_under_sanitizers(tmp_path):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "oracle_checks")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", os.path.join(ROOT, "tests", "sanitize", "oracle_checks.cpp"), "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle checks passed" in r.stdout


def test_library_host_code_under_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not found")
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-sanitize-recover=all",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    jobs = [[HIPCC, *flags, "-c", os.path.join(CSRC, f + ".hip"), "-o", str(tmp_path / (f + ".o"))]
            for f in SOURCES]
    jobs.append([HIPCC, *flags, "-x", "hip", "-c", os.path.join(ROOT, "tests", "sanitize", "host_checks.cpp"),
                 "-o", str(tmp_path / "host_checks.o")])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as pool:
        list(pool.map(_run, jobs))
    exe = str(tmp_path / "host_checks")
    objs = [str(tmp_path / (f + ".o")) for f in SOURCES] + [str(tmp_path / "host_checks.o")]
    _run([HIPCC, "--offload-arch=gfx950", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          *objs, "-o", exe])
    syms = _run(["nm", exe]).stdout
    assert "__asan_report" in syms and "__ubsan_handle" in syms   # the host code is instrumented
    r = _run([exe], env=ENV, timeout=300)
    assert "host checks passed" in r.stdout
