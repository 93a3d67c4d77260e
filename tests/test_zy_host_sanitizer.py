"""GPU: the library's host code under AddressSanitizer.

tests/native/abi_sanitized.cpp drives the C ABI through its main paths (every
incident-field kind, the three precisions and table layouts, host results, the
time transform, a batch, evaluation without allocation, the tuner, error
returns, and a serving loop fed from two client threads with cancellations and
a shutdown with requests still queued).  `build()` links it with the library's
sources into tests/native/_build/abi_address, the host code instrumented (the
gfx950 kernels are the library's own).  A heap overflow, use after free, double
free or leak of the library's own allocations (the ROCm runtime's own, held
until the process ends, are suppressed by tests/native/lsan_rocm.supp) ends
the run with a sanitizer report and a non-zero status.  (ThreadSanitizer is not
used: under its fixed shadow-memory layout the ROCm runtime finds no device.)
The file is named to be collected after the other GPU tests but before the
no-allocation test.
"""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "native", "_build")


def test_abi_paths_under_address_sanitizer():
    exe = os.path.join(BUILD, "abi_address")
    if not os.path.exists(exe):
        pytest.skip(f"{exe} is not built (the repository build step builds it)")
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    env["LSAN_OPTIONS"] = "suppressions=" + os.path.join(HERE, "native", "lsan_rocm.supp")
    print(f"running {exe}", flush=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout[-2000:], r.stderr[-6000:], flush=True)
    assert r.returncode == 0, r.stderr[-6000:]
    assert "clean under the sanitizer" in r.stdout
