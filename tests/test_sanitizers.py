"""The host code under AddressSanitizer and UndefinedBehaviorSanitizer, and
the serving scheduler under ThreadSanitizer (CPU only).

- The oracle (orc.c, gcc) and the library's host-only sources (region
  polygons, drift map; g++) are rebuilt with -fsanitize=address,undefined
  and the CPU tests that exercise them run in a child process with the ASan
  runtime preloaded; any report fails the test.
- The serving runtime, built host-only (no device code) with
  -fsanitize=thread, runs its dry-run scheduler under concurrent submitters
  and pollers in a small driver program; any race report fails the test.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2411_01919_amd", "csrc")


def _gcc_runtime(name):
    p = subprocess.check_output(["gcc", f"-print-file-name={name}"]).decode().strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(shutil.which("gcc") is None or shutil.which("g++") is None, reason="needs gcc")
def test_host_code_under_asan_and_ubsan(tmp_path):
    asan = _gcc_runtime("libasan.so")
    if asan is None:
        pytest.skip("no libasan")
    san = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    orc = tmp_path / "liborc_san.so"
    subprocess.check_call(["gcc", *san, "-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
                           os.path.join(ROOT, "oracle", "orc.c"), "-o", str(orc), "-lm"])
    host = tmp_path / "libpphost_san.so"
    subprocess.check_call(["g++", *san, "-std=c++17", "-fPIC", "-shared", "-I", os.path.join(ROOT, "include"),
                           os.path.join(CSRC, "pp_polygons.cpp"), os.path.join(CSRC, "pp_map.cpp"), "-o", str(host)])
    env = dict(os.environ, LD_PRELOAD=asan, ORC_LIB=str(orc), PP_HOST_SAN_LIB=str(host), OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    files = ["tests/test_oracle_diffusion.py", "tests/test_oracle_diffusion_variants.py",
             "tests/test_oracle_normals.py", "tests/test_oracle_valid_list.py", "tests/test_oracle_philox.py",
             "tests/test_oracle_ransac.py", "tests/test_oracle_regions.py", "tests/test_oracle_segment.py",
             "tests/test_oracle_polygons.py", "tests/test_polygons.py", "tests/test_map.py", "tests/test_golden.py"]
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "san_child.py"), *files], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out


def _clang_tsan():
    hipcc = "/opt/rocm/bin/hipcc"
    return hipcc if os.path.exists(hipcc) else None


@pytest.mark.skipif(_clang_tsan() is None, reason="needs hipcc")
def test_scheduler_under_tsan(tmp_path):
    """Several submitter threads and a poller thread against the dry-run
    scheduler (admission under a tight budget, two lanes, a stream closed
    while it has queued frames); ThreadSanitizer must report nothing."""
    hipcc = _clang_tsan()
    exe = tmp_path / "server_tsan"
    srcs = [os.path.join(CSRC, s) for s in ("pp_server.hip", "pp_api.hip", "pp_kernels.hip", "pp_regions.hip",
                                            "pp_segment.hip")]
    srcs += [os.path.join(CSRC, "pp_polygons.cpp"), os.path.join(CSRC, "pp_map.cpp")]
    # the sanitizer applies to the host side only (-Xarch_host); device code builds as usual
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-Xarch_host", "-fsanitize=thread",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs,
           os.path.join(ROOT, "tests", "native", "server_tsan.cpp"), "-o", str(exe), "-lpthread"]
    subprocess.check_call(cmd, cwd=tmp_path)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1")
    r = subprocess.run([str(exe)], env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert "ThreadSanitizer" not in out, out[-4000:]
    assert r.returncode == 0 and "server_tsan ok" in out, out[-4000:]
