"""The definition of g(E, M) vectorised with numpy, for small N (<= 22).

Test infrastructure only.  Follows Section 2, Eq. (1): every configuration
(bit u set means s_u = +1) gets E = -sum_b J_b s_i s_j and n_up = number of
up spins; g counts configurations per (E, n_up).  Used to cross-check the C
brute force, which implements the same definition with plain loops.
"""
from __future__ import annotations

import numpy as np


def g_numpy(n_spins: int, bond_i, bond_j, bond_J) -> np.ndarray:
    if n_spins > 22:
        raise ValueError("g_numpy is for small systems only")
    bond_i = np.asarray(bond_i, dtype=np.int64)
    bond_j = np.asarray(bond_j, dtype=np.int64)
    bond_J = np.asarray(bond_J, dtype=np.int64)
    S = int(np.abs(bond_J).sum())
    c = np.arange(1 << n_spins, dtype=np.int64)
    s = ((c[:, None] >> np.arange(n_spins)[None, :]) & 1) * 2 - 1  # [2^N, N] spins
    E = -(s[:, bond_i] * s[:, bond_j] * bond_J[None, :]).sum(axis=1)
    n_up = ((s + 1) // 2).sum(axis=1)
    g = np.zeros((2 * S + 1, n_spins + 1), dtype=np.uint64)
    np.add.at(g, (E + S, n_up), 1)
    return g
