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


# binding structure -> C typedef in include/geneo.h
_STRUCTS = {"Mesh": "geneo_mesh", "SystemInfo": "geneo_system_info", "PartitionOpts": "geneo_partition_opts",
            "DecompInfo": "geneo_decomp_info", "SetupOpts": "geneo_setup_opts",
            "PrecondInfo": "geneo_precond_info", "ModelOpts": "geneo_model_opts", "ModelInfo": "geneo_model_info",
            "TrainOpts": "geneo_train_opts", "TrainInfo": "geneo_train_info",
            "FactorSchedule": "geneo_factor_schedule", "SolveOpts": "geneo_solve_opts",
            "SolveInfo": "geneo_solve_info"}


def test_binding_structures_match_the_header(tmp_path):
    """Every ctypes structure of the binding has the size and field offsets
    of its C typedef, as the host C compiler lays it out from the header: a
    field added to one side only would shift every later field."""
    import shutil
    import subprocess
    from paper_2311_18783_amd import geneo
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "geneo.h"', "int main(void) {"]
    expect = []
    for py, c in _STRUCTS.items():
        cls = getattr(geneo, py)
        lines.append(f'  printf("%zu\\n", sizeof({c}));')
        expect.append((f"sizeof {c}", ctypes.sizeof(cls)))
        for f in cls._fields_:
            lines.append(f'  printf("%zu\\n", offsetof({c}, {f[0]}));')
            expect.append((f"{c}.{f[0]}", getattr(cls, f[0]).offset))
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert len(got) == len(expect)
    bad = [(name, want, g) for (name, want), g in zip(expect, got) if want != g]
    assert not bad, bad
