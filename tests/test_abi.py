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


@pytest.mark.skipif(not os.path.exists(LIB), reason="libgeneo.so not built")
def test_binding_rejects_bad_vectors_before_the_library():
    """Device vectors are checked in the binding before any library call: a
    host tensor, a float32 tensor, a strided view or a wrong length raises
    ValueError, so no kernel ever sees a buffer of the wrong size or type."""
    import torch
    from paper_2311_18783_amd import geneo
    with pytest.raises(ValueError, match="device|cuda"):
        geneo.check_vector(torch.zeros(10, dtype=torch.float64), 10, 0)
    with pytest.raises(ValueError, match="dtype"):
        geneo.check_vector(torch.zeros(10, dtype=torch.float32), 10, 0)
    with pytest.raises(ValueError, match="tensor"):
        geneo.check_vector(list(range(10)), 10, 0)
    with pytest.raises(ValueError, match="contiguous"):
        geneo.check_vector(torch.zeros(20, dtype=torch.float64)[::2], 10, 0)
    with pytest.raises(ValueError, match="elements"):
        geneo.check_vector(torch.zeros(9, dtype=torch.float64), 10, 0)
