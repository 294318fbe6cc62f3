"""The C-ABI library loads and exports every symbol the header declares (no GPU)."""
import ctypes
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2311_18783_amd", "libgeneo.so")


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgeneo.so not built")
def test_library_exports_header_symbols():
    from paper_2311_18783_amd import geneo
    names = geneo.header_symbols()
    assert len(names) >= 20
    lib = ctypes.CDLL(LIB)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgeneo.so not built")
def test_null_arguments_rejected_without_device():
    from paper_2311_18783_amd import geneo
    assert geneo.lib.geneo_create(None, 0, None) == -1
    assert geneo.lib.geneo_assemble(None, None, None, None, 1.0, None) == -1
    assert geneo.lib.geneo_solve(None, None, None, None, None, None, None) == -1
