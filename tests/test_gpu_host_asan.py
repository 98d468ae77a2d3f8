"""The library's host code under AddressSanitizer (device code unchanged):
tests/asan/host_driver, built by tests/asan/build_asan.py against a host-ASan
build of libsbci, drives every entry point on small cases (unblocked shapes
including an empty spin and Sz != 0, a point-group blocked context, sigma in
three dtypes, the three precision forms, Davidson, SBCI2, the step interface,
refusals, the trace, and a batch with its tuner, BF16 solve and vector export).
It must end with no sanitizer report; leaks inside the ROCm runtime libraries
are suppressed (tests/asan/lsan.supp)."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.join(os.path.dirname(__file__), "asan")


def test_host_code_clean_under_asan():
    exe = os.path.join(HERE, "host_driver")
    assert os.path.exists(exe), "tests/asan/host_driver is not built (run __graft_entry__.build())"
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               LSAN_OPTIONS="suppressions=" + os.path.join(HERE, "lsan.supp"))
    print("host ASan driver", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "ALL_OK" in r.stdout, out[-3000:]
    assert "ERROR: AddressSanitizer" not in out and "ERROR: LeakSanitizer" not in out, out[-3000:]
