"""The CPU oracle against its pins (no GPU)."""
import pytest

import oracle
import pins


@pytest.fixture(scope="module")
def orc():
    return oracle.load()


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)


def test_oracle_rejects_bad_arguments(orc):
    import numpy as np

    lib = orc.lib
    k = np.zeros(4, dtype=np.uint32)
    assert lib.orc_sort(7, 0, 0, 0, k.ctypes.data, None, None, 4) == -4      # unknown algorithm
    assert lib.orc_sort(0, 9, 0, 0, k.ctypes.data, None, None, 4) == -3      # unknown dtype
    assert lib.orc_sort(0, 0, 1 << 9, 0, k.ctypes.data, None, None, 4) == -4  # network of size 9
    assert lib.orc_sort(0, 0, 0, 0, None, None, None, 4) == -1
    assert lib.orc_sort(0, 0, 0, 0, k.ctypes.data, None, None, -1) == -2
    off = np.array([0, 3, 2, 4], dtype=np.uint32)                            # decreasing offsets
    assert lib.orc_segmented_sort(0, 0, 0, 0, k.ctypes.data, None, None, off.ctypes.data, 3) == -2
    g = np.zeros((1, 4), dtype=np.float32)
    p = np.array([[0, 1, 2, 4]], dtype=np.int32)                             # index out of row
    assert lib.orc_gather_backward(g.ctypes.data, p.ctypes.data, g.ctypes.data, 1, 4) == -2
