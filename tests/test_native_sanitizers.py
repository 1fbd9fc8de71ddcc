"""Host-code checks under the sanitizers (CPU only, no GPU).

- The batch scheduler of hgp_run_jobs (paper_2605_20497_amd/csrc/hgp_batch.cpp),
  compiled with g++ against a host stand-in of its two HIP runtime calls and
  of the context calls (tests/native/), runs hundreds of jobs with staggered
  arrivals on 8 and 16 workers under ThreadSanitizer, and again under
  AddressSanitizer + UndefinedBehaviorSanitizer.
- The serial oracle runs a randomised driver through every C entry point
  under AddressSanitizer + UndefinedBehaviorSanitizer.
A report from any sanitizer fails the test.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN_MARKERS = ("WARNING: ThreadSanitizer", "ERROR: AddressSanitizer", "ERROR: LeakSanitizer", "runtime error:")


def _build_run(tmp_path, name, sources, flags, args=(), env=None):
    exe = str(tmp_path / name)
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", "-I" + os.path.join(NATIVE, "hip_stub")] + flags + \
        ["-o", exe] + sources
    subprocess.check_call(cmd)
    r = subprocess.run([exe] + [str(a) for a in args], capture_output=True, text=True, timeout=600,
                       env=dict(os.environ, **(env or {})))
    out = r.stdout + r.stderr
    for m in SAN_MARKERS:
        assert m not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    return out


BATCH = [os.path.join(ROOT, "paper_2605_20497_amd", "csrc", "hgp_batch.cpp"),
         os.path.join(NATIVE, "batch_stub_api.cpp"), os.path.join(NATIVE, "batch_driver.cpp")]


@pytest.mark.parametrize("workers", [8, 16])
def test_batch_scheduler_tsan(tmp_path, workers):
    out = _build_run(tmp_path, "batch_tsan", BATCH, ["-fsanitize=thread"], (300, workers),
                     env={"TSAN_OPTIONS": "halt_on_error=1"})
    assert "bad 0" in out
    assert "put back 0 " not in out  # the put-back path ran


def test_batch_scheduler_asan_ubsan(tmp_path):
    out = _build_run(tmp_path, "batch_asan", BATCH, ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                     (300, 8), env={"ASAN_OPTIONS": "detect_leaks=1"})
    assert "bad 0" in out


def test_oracle_asan_ubsan(tmp_path):
    out = _build_run(tmp_path, "oracle_asan", [os.path.join(NATIVE, "oracle_driver.cpp")],
                     ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
                     env={"ASAN_OPTIONS": "detect_leaks=1"})
    assert "bad 0" in out
