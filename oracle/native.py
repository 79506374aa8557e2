"""Build and load the C part of the oracle (oracle.c) with gcc, via ctypes.

Test infrastructure only: see the package docstring.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so (plain C, gcc -O2 with the x86-64 popcount instruction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-mpopcnt", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True)
            lib = ctypes.CDLL(_LIB)
            i32p = ctypes.POINTER(ctypes.c_int32)
            u64p = ctypes.POINTER(ctypes.c_uint64)
            lib.oracle_count_range.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p,
                                               ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int, u64p]
            lib.oracle_count_range.restype = ctypes.c_int
            lib.oracle_tm_torus.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, ctypes.c_int, u64p]
            lib.oracle_tm_torus.restype = ctypes.c_int
            lib.oracle_bond_split.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, ctypes.c_int,
                                              u64p, u64p]
            lib.oracle_bond_split.restype = ctypes.c_int
            lib.oracle_band_count.argtypes = [ctypes.c_int, ctypes.c_int, i32p, i32p, i32p, u64p]
            lib.oracle_band_count.restype = ctypes.c_int
            lib.oracle_row_words.argtypes = [ctypes.c_int, ctypes.c_int, u64p, u64p, ctypes.c_uint64,
                                             ctypes.c_uint64, ctypes.c_int, u64p]
            lib.oracle_row_words.restype = ctypes.c_int
            _lib = lib
        return _lib


def default_threads() -> int:
    """Host threads to use: the CPUs this process may run on, at most 16."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _i32(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int32))
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def count_range(n_spins: int, bond_i, bond_j, bond_J, first: int, count: int,
                n_threads: int | None = None) -> np.ndarray:
    """g over configurations with index in [first, first+count): uint64 [2S+1][N+1]."""
    lib = _load()
    bi, pbi = _i32(bond_i)
    bj, pbj = _i32(bond_j)
    bJ, pbJ = _i32(bond_J)
    S = int(np.abs(bJ.astype(np.int64)).sum())
    g = np.zeros((2 * S + 1, n_spins + 1), dtype=np.uint64)
    rc = lib.oracle_count_range(int(n_spins), int(bi.shape[0]), pbi, pbj, pbJ,
                                int(first), int(count), int(n_threads or default_threads()),
                                g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError(f"oracle_count_range failed ({rc})")
    return g


def count_all(n_spins: int, bond_i, bond_j, bond_J, n_threads: int | None = None) -> np.ndarray:
    """g(E, M) of all 2^N configurations (the definition, brute force)."""
    return count_range(n_spins, bond_i, bond_j, bond_J, 0, 1 << n_spins, n_threads)


def tm_torus(Jh, Jv, n_threads: int | None = None) -> np.ndarray:
    """Exact g of a square torus from the transfer matrix: uint64 [2S+1][N+1].

    Jh, Jv: int [Ly][Lx] coupling grids (see oracle.c for the bond geometry).
    """
    lib = _load()
    Jh = np.asarray(Jh, dtype=np.int32)
    Jv = np.asarray(Jv, dtype=np.int32)
    if Jv.shape != Jh.shape:
        raise ValueError("Jh and Jv must have the same shape")
    if Jh.shape[1] > Jh.shape[0]:
        # Transfer along the longer side: the transposed torus (rows <-> columns,
        # horizontal <-> vertical bonds) is the same graph with sites renamed,
        # so its g is identical and the row states are fewer.
        Jh, Jv = Jv.T, Jh.T
    Jh, pJh = _i32(Jh)
    Jv, pJv = _i32(Jv)
    Ly, Lx = Jh.shape
    S = int(np.abs(Jh.astype(np.int64)).sum() + np.abs(Jv.astype(np.int64)).sum())
    g = np.zeros((2 * S + 1, Lx * Ly + 1), dtype=np.uint64)
    rc = lib.oracle_tm_torus(int(Lx), int(Ly), pJh, pJv, int(n_threads or default_threads()),
                             g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError(f"oracle_tm_torus failed ({rc})")
    return g


def row_words(Lx: int, Ly: int, first: int = 0, count: int | None = None,
              n_threads: int | None = None, Jh=None, Jv=None) -> np.ndarray:
    """g of the Lx x Ly square torus with couplings +-1 by the paper's bit-word
    scheme (Section 3), over configurations [first, first + count) (default
    all): uint64 [4N+1][N+1], row E + 2N, column n_up.  Jh, Jv are the
    [Ly][Lx] coupling grids of lattice.torus_coupling_grids (entries +-1;
    default all 1): Jh[y][x] couples (x, y)-(x+1, y), Jv[y][x] couples
    (x, y)-(x, y+1).  A J = -1 bond is satisfied when its spins differ, which
    the scheme handles with one more XOR against a per-row sign mask."""
    lib = _load()
    N = Lx * Ly
    count = (1 << N) - first if count is None else count
    masks = []
    for grid in (Jh, Jv):
        m = np.zeros(max(Ly, 1), dtype=np.uint64)
        if grid is not None:
            grid = np.asarray(grid, dtype=np.int64)
            if grid.shape != (Ly, Lx) or not np.isin(grid, (-1, 1)).all():
                raise ValueError("coupling grids must be [Ly][Lx] with entries +-1")
            for y in range(Ly):
                m[y] = sum(1 << x for x in range(Lx) if grid[y, x] < 0)
        masks.append(m)
    g = np.zeros((4 * N + 1, N + 1), dtype=np.uint64)
    pu = ctypes.POINTER(ctypes.c_uint64)
    rc = lib.oracle_row_words(int(Lx), int(Ly), masks[0].ctypes.data_as(pu), masks[1].ctypes.data_as(pu),
                              int(first), int(count), int(n_threads or default_threads()), g.ctypes.data_as(pu))
    if rc != 0:
        raise ValueError(f"oracle_row_words failed ({rc})")
    return g


def band_count(n_spins: int, bond_i, bond_j, bond_J) -> np.ndarray:
    """Exact g by the banded count along the site order (oracle.c), for
    lattices whose bonds join sites at most 20 apart: uint64 [2S+1][N+1]."""
    lib = _load()
    bi, pbi = _i32(bond_i)
    bj, pbj = _i32(bond_j)
    bJ, pbJ = _i32(bond_J)
    S = int(np.abs(bJ.astype(np.int64)).sum())
    g = np.zeros((2 * S + 1, n_spins + 1), dtype=np.uint64)
    rc = lib.oracle_band_count(int(n_spins), int(bi.shape[0]), pbi, pbj, pbJ,
                               g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError(f"oracle_band_count failed ({rc})")
    return g


def bond_split(n_spins: int, bond_i, bond_j, bond_J, n_threads: int | None = None):
    """(g, gp): g as count_all, and gp [n_bonds][2S+1][N+1] with gp[b][E][n_up]
    the number of configurations in that bin whose bond-b spins agree."""
    lib = _load()
    bi, pbi = _i32(bond_i)
    bj, pbj = _i32(bond_j)
    bJ, pbJ = _i32(bond_J)
    S = int(np.abs(bJ.astype(np.int64)).sum())
    nb = int(bi.shape[0])
    g = np.zeros((2 * S + 1, n_spins + 1), dtype=np.uint64)
    gp = np.zeros((max(nb, 1), 2 * S + 1, n_spins + 1), dtype=np.uint64)
    rc = lib.oracle_bond_split(int(n_spins), nb, pbi, pbj, pbJ, int(n_threads or default_threads()),
                               g.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               gp.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)))
    if rc != 0:
        raise ValueError(f"oracle_bond_split failed ({rc})")
    return g, gp[:nb]


def tm_torus_bond_split(Jh, Jv, direction: int, x: int, y: int, n_threads: int | None = None):
    """(g, gp) of one bond of a square torus from the transfer matrix, for
    tori too large for bond_split's brute force.

    The bond couples (x, y) to (x+1, y) when direction is 0 (coupling Jh[y][x])
    and to (x, y+1) when it is 1 (Jv[y][x]).  Eq. (1) makes H depend on the
    bond's coupling J_b only through -J_b s_i s_j, so raising J_b by D > 2S
    moves every configuration with s_i s_j = +1 from E to E - D < -S and every
    one with s_i s_j = -1 to E + D > S: the shifted torus's table holds the two
    halves apart, each an exact copy of its part of g.  g[E + S][n_up] is the
    unshifted table, gp its part with s_i s_j = +1 (as bond_split).
    """
    Jh = np.array(Jh, dtype=np.int64)
    Jv = np.array(Jv, dtype=np.int64)
    S = int(np.abs(Jh).sum() + np.abs(Jv).sum())
    D = 2 * S + 1
    grid = Jh if direction == 0 else Jv
    Jb = int(grid[y, x])
    grid[y, x] = Jb + D
    S2 = S - abs(Jb) + abs(Jb + D)
    g2 = tm_torus(Jh, Jv, n_threads)
    # rows of E' in [-S - D, S + D] (the shifted table spans only [-S2, S2])
    pad = S + D - S2
    g2 = np.concatenate([np.zeros((pad, g2.shape[1]), np.uint64), g2, np.zeros((pad, g2.shape[1]), np.uint64)])
    ne = 2 * S + 1
    lo = 0              # row of E' = E - D for E = -S: configurations with s_i s_j = +1
    hi = 2 * D          # row of E' = E + D for E = -S: configurations with s_i s_j = -1
    gp = g2[lo:lo + ne].copy()
    gm = g2[hi:hi + ne].copy()
    rest = g2.copy()
    rest[lo:lo + ne] = 0
    rest[hi:hi + ne] = 0
    if rest.any():
        raise AssertionError("shifted bond left counts outside its two energy windows")
    return gp + gm, gp
