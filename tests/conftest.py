import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: takes more than a few seconds on the CPU")


def load_table1():
    """Table 1 of the paper as {(E, M): count}."""
    path = os.path.join(ROOT, "tests", "golden", "table1_4x4.txt")
    out = {}
    with open(path) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            nc, m, e = (int(v) for v in line.split())
            assert (e, m) not in out
            out[(e, m)] = nc
    return out


def nonzero_bins(g, e_min, n_spins):
    """Dense g[E - e_min][n_up] -> {(E, M): count} over nonzero bins."""
    import numpy as np
    e_idx, n_up = np.nonzero(g)
    return {(int(e) + e_min, 2 * int(n) - n_spins): int(g[e, n]) for e, n in zip(e_idx, n_up)}
