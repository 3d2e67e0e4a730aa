"""The host side under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only):

* the library's host code (argument checks, workspace planning, weight
  packing, every entry point's control flow), built with g++ against a
  host-only stand-in for the HIP runtime whose kernel launchers only count
  (tests/hostbuild/): every LNM_ERR_* path a caller can reach returns its
  status, sets an error message and launches nothing, and valid calls launch;
* every function of the fp64 oracle on small ragged inputs.

LNM_ERR_OOM (a failed host allocation) cannot be reached through arguments
and is not exercised."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HB = os.path.join(ROOT, "tests", "hostbuild")
CSRC = os.path.join(ROOT, "paper_2604_03748_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_library_host_code_error_paths_under_sanitizers(tmp_path):
    exe = str(tmp_path / "check_host")
    sources = [os.path.join(CSRC, f) for f in ("api.hip", "plan.hip", "train_api.hip", "frame_static.hip")]
    _run(["g++", "-std=c++17", *SAN, f"-I{HB}", f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}", "-x", "c++",
          *sources, "-x", "none", os.path.join(HB, "fake_device.cpp"), os.path.join(HB, "check_host.cpp"), "-o", exe])
    r = _run([exe], env=ENV)
    assert " 0 failures" in r.stdout, r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "check_oracle")
    _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp", *SAN,
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HB, "check_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV)
    assert "0 failures" in r.stdout, r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
