"""Host-only runtime pieces built with AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU (no GPU):

  * tests/native/arena_admit_test.cpp: the budgeted sub-allocator behind
    every device allocation of a context (fake device chunks from malloc:
    first fit, top placement, coalescing, shrink, budget, chunk release,
    allocator failures, randomised operation sequences against a model, 8
    threads) and the scheduler's FIFO admission rule against a fake executor
    with its own memory budget (order, no starvation, requests too large for
    the budget, errors, slot limits);
  * tests/native/lossless_test.cpp: the lossless coder's entry points (round
    trips for both codecs with and without the shuffle; truncated, flipped,
    forged and random input must end in an error code).
"""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_20731_amd", "csrc")
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
       "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def _build_and_run(tmp_path, name, srcs, extra=(), libs=()):
    exe = str(tmp_path / name)
    cmd = ["g++", *SAN, *extra, "-I", CSRC, "-I", os.path.join(ROOT, "include"), *srcs, "-o", exe, *libs]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0 and "ALL OK" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    return r.stdout


def test_arena_and_admission_sanitized(tmp_path):
    _build_and_run(tmp_path, "arena_admit", [os.path.join(NATIVE, "arena_admit_test.cpp"),
                                             os.path.join(CSRC, "isr_arena.cpp")], libs=["-lpthread"])


@pytest.mark.skipif(not os.path.exists("/opt/rocm/lib/libamdhip64.so"), reason="HIP runtime library not present")
def test_lossless_coder_sanitized(tmp_path):
    out = _build_and_run(tmp_path, "lossless", [os.path.join(NATIVE, "lossless_test.cpp"),
                                               os.path.join(CSRC, "isr_lossless.cpp")],
                         extra=["-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"],
                         libs=["-L/opt/rocm/lib", "-lamdhip64", "-lz", "-l:libbz2.so.1", "-lpthread",
                               "-Wl,-rpath,/opt/rocm/lib"])
    assert "rejected" in out
