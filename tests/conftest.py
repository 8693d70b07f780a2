import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: long-running case")


def matrix_from_upper(n, entries, fill_lower=np.nan):
    """n x n fp32 matrix from [a, b, value] strict-upper entries; the lower
    triangle and diagonal get ``fill_lower`` (they must be ignored)."""
    d = np.full((n, n), fill_lower, dtype=np.float32)
    for a, b, v in entries:
        d[a, b] = v
    return d
