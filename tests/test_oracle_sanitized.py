"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/native/oracle_sanitized.c calls every oracle entry point on small inputs in
buffers of exactly the documented sizes; built together with oracle/sc_oracle.c
with -fsanitize=address,undefined (and no recovery), any out-of-bounds access,
use after free, leak or undefined operation in the oracle ends the run with an
error, which fails this test.  (The planted-overrun check below shows that the
build does catch one.)
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
DRIVER = os.path.join(HERE, "native", "oracle_sanitized.c")
ORACLE = os.path.join(ROOT, "oracle", "sc_oracle.c")
FLAGS = ["-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-fopenmp"]


def _build(src, out):
    subprocess.check_call(["gcc", *FLAGS, "-o", out, src, ORACLE, "-lquadmath", "-lm"])


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)


@pytest.fixture(scope="module")
def workdir(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    return tmp_path_factory.mktemp("sanitized")


def test_oracle_entry_points_are_clean(workdir):
    exe = str(workdir / "oracle_sanitized")
    _build(DRIVER, exe)
    r = _run(exe)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "clean under the sanitizers" in r.stdout


def test_the_sanitized_build_catches_an_overrun(workdir):
    """The same driver with one call told of one point more than its buffers hold."""
    src = open(DRIVER).read()
    call = "orc_incident_lg(2, pl, exy, 1.5, n_tot, pos, kv[0], 1.0, 0.0, El, Bl);"
    assert call in src
    bad = workdir / "oracle_overrun.c"
    bad.write_text(src.replace(call, call.replace("n_tot, pos", "n_tot + 1, pos")))
    exe = str(workdir / "oracle_overrun")
    _build(str(bad), exe)
    r = _run(exe)
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr
