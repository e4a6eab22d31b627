"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two programs are built and run on ragged and degenerate patterns:
- tests/sanitize/oracle_main.c with the FP64 oracle (gcc);
- tests/sanitize/host_planners.cpp with the HIP library's host-side
  planners: the workspace plan, the gather layout's workgroup blocking, the
  binned layout's blocking and host-built tile tables, the batched tiling and
  host validation.  hipcc builds it; the sanitizers apply to the host code
  only (each -fsanitize= behind -Xarch_host) and the program makes no GPU
  call, so it runs without a GPU.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2509_10722_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LINKED = ["pmp_kernels.hip", "pmp_binned.hip", "pmp_binned_plan.hip", "pmp_adjoint.hip",
          "pmp_prune.hip"]   # pmp_api.hip and pmp_batch.hip are included by the harness
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, env=None, timeout=600):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=timeout, env=env)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    _run(["gcc", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "oracle_main.c"),
          os.path.join(ROOT, "oracle", "pmp_oracle.c"), "-lm"])
    r = _run([exe], env=ENV)
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_host_planners_under_sanitizers(tmp_path):
    exe = str(tmp_path / "planners_asan")
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-sanitize-recover=all",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-x", "hip",
          os.path.join(HERE, "host_planners.cpp"), *[os.path.join(CSRC, f) for f in LINKED],
          "-o", exe], timeout=900)
    # the HIP runtime keeps process-lifetime allocations: no leak report
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0"))
    assert "all checks passed" in r.stdout
    assert "runtime error" not in r.stderr
