"""The autotuner's schedule table (host only, no GPU): text round trip,
lookup by key with the nearest-block fallback, defaults, bad input."""
import os
import tempfile

import numpy as np
import pytest

from paper_2311_18783_amd import geneo


def _write(txt):
    fd, path = tempfile.mkstemp(suffix=".txt")
    with os.fdopen(fd, "w") as f:
        f.write(txt)
    return path


def test_defaults_without_entries():
    # a key no test below writes: precision FP64, 1000 block columns, class 9
    assert geneo.tune_lookup([128000] * 600, geneo.FP64) == (0, 8, 1)


def test_load_lookup_nearest_and_roundtrip():
    # FP32, class 6 (64..127 matrices): entries at 10 and 30 block columns
    path = _write("# comment\n1 10 6 2 4 0 1.5\n1 30 6 1 16 0 2.5\n")
    try:
        geneo.tune_load(path)
    finally:
        os.unlink(path)
    sizes = lambda nb, m: [nb * 128] * m
    assert geneo.tune_lookup(sizes(10, 64), geneo.FP32_REFINE1) == (2, 4, 0)
    assert geneo.tune_lookup(sizes(30, 100), geneo.FP32_REFINE1) == (1, 16, 0)
    # nearest tuned block count within the same precision and class
    assert geneo.tune_lookup(sizes(12, 70), geneo.FP32_REFINE1) == (2, 4, 0)
    assert geneo.tune_lookup(sizes(27, 70), geneo.FP32_REFINE1) == (1, 16, 0)
    # another class or precision does not see them
    assert geneo.tune_lookup(sizes(10, 8), geneo.FP32_REFINE1) == (0, 8, 1)
    fd, out = tempfile.mkstemp(suffix=".txt")
    os.close(fd)
    try:
        geneo.tune_save(out)
        lines = [l.split() for l in open(out) if not l.startswith("#")]
    finally:
        os.unlink(out)
    assert ["1", "10", "6", "2", "4", "0"] in [l[:6] for l in lines]
    assert ["1", "30", "6", "1", "16", "0"] in [l[:6] for l in lines]


@pytest.mark.parametrize("bad", ["1 10 6 3 4 0 1.0\n", "2 10 6 0 4 0 1.0\n", "0 0 6 0 4 1 1.0\n",
                                 "0 10 6 0 0 1 1.0\n", "0 10 6 0 4 2 1.0\n", "0 10 six 0 4 1 1.0\n"])
def test_bad_lines_are_rejected_and_change_nothing(bad):
    path = _write("0 5 3 1 4 1 1.0\n" + bad)
    try:
        with pytest.raises(geneo.GeneoError):
            geneo.tune_load(path)
    finally:
        os.unlink(path)
    # the good line before the bad one was not merged either
    assert geneo.tune_lookup([5 * 128] * 8, geneo.FP64) == (0, 8, 1)


def test_missing_file():
    with pytest.raises(geneo.GeneoError):
        geneo.tune_load("/nonexistent/table.txt")
