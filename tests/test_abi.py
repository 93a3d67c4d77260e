"""The C-ABI library builds for gfx950, loads, and exports every entry point
declared in include/sc.h (no GPU needed: no compute calls are made)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sc.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:sc_status|const char\s*\*)\s*(sc_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1609_08146_amd import _abi
    if not os.path.exists(_abi.LIB_PATH):
        from paper_1609_08146_amd import build
        build.build()
    return ctypes.CDLL(_abi.LIB_PATH)


def test_header_declares_the_path():
    syms = declared_symbols()
    for name in ["sc_ctx_create", "sc_set_mirror", "sc_set_frequencies", "sc_set_incident",
                 "sc_set_incident_gaussian", "sc_set_observation", "sc_evaluate", "sc_to_time",
                 "sc_evaluate_batch", "sc_server_create", "sc_server_submit", "sc_server_wait"]:
        assert name in syms


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    from paper_1609_08146_amd import _abi
    assert sorted(_abi.SIGNATURES) == declared_symbols()


def test_library_is_gfx950_code_object(lib):
    from paper_1609_08146_amd import _abi
    data = open(_abi.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_version_and_error_strings(lib):
    from paper_1609_08146_amd import _abi
    lib2 = _abi.load()
    assert b"gfx950" in lib2.sc_version()
    # argument validation happens before any device work
    assert lib2.sc_ctx_create(0, None, None) == _abi.SC_E_INVAL
    assert b"NULL" in lib2.sc_last_error()
    assert lib2.sc_set_mirror(None, 1.0, 1.0, 1, 1) == _abi.SC_E_INVAL


def test_binding_fails_loudly_without_library(tmp_path):
    import subprocess
    import sys
    code = ("import os; os.environ['SC_LIBRARY']=r'%s';\n"
            "from paper_1609_08146_amd import _abi\n"
            "try:\n    _abi.load()\nexcept ImportError as e:\n    print('IMPORTERROR', e)\n") % (tmp_path / "none.so")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert "IMPORTERROR" in out.stdout
