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


def load_cube_goldens():
    """{member index: dense uint64 table} of the 3x3x3 cubes of the batch256
    workload, as the oracle's brute force counted them
    (tests/golden/make_batch256_cubes.py).  Each entry is checked to belong to
    the workload's lattice by its coupling seed and a SHA-256 of its bonds."""
    import hashlib

    import numpy as np

    from paper_1110_2561_amd import lattice as L
    z = np.load(os.path.join(ROOT, "tests", "golden", "batch256_cubes.npz"))
    lats = L.workload("batch256")["lattices"]
    out = {}
    for c, i in enumerate(z["member"].tolist()):
        lat = lats[i]
        h = hashlib.sha256()
        for a in (lat.bond_i, lat.bond_j, lat.bond_J):
            h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
        assert lat.kind == "cubic_torus" and int(z["seed"][c]) == lat.seed, f"member {i}"
        assert z["bonds_sha"][c].decode() == h.hexdigest(), f"member {i}: lattice differs from the golden's"
        g = np.zeros((int(z["n_e"][c]), lat.n_spins + 1), dtype=np.uint64)
        a, b = int(z["offsets"][c]), int(z["offsets"][c + 1])
        g[z["e_idx"][a:b].astype(np.int64), z["n_up"][a:b].astype(np.int64)] = z["count"][a:b]
        out[i] = g
    return out


def moment_scales(g, S, N, T, h):
    """The oracle's moments of a table on a (T, h) grid, and for each
    derivative of log Z the magnitude of the terms its formula sums or
    subtracts (a forward error bound is a small multiple of eps times it):
      d_T  = <H>/T^2               |H| <= S + |h| N
      d_h  = <M>/T                 |M| <= N
      d_TT = Var(H)/T^4 - 2<H>/T^3
      d_Th = (Cov(H, M)/T - <M>)/T^2,  |Cov| <= sqrt(Var(H) Var(M))
      d_hh = Var(M)/T^2
    Keys: mE, mM, mH, C, chi (oracle values) and d_T .. d_hh (scales)."""
    import numpy as np

    from oracle import thermo
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    mE, mM, C, chi = thermo.moments(g, -S, N, T, h)
    Tc, hr = T[:, None], h[None, :]
    varH, varM = C * Tc * Tc, chi * Tc
    hmax = S + np.abs(hr) * N + 0 * Tc
    return {"mE": mE, "mM": mM, "C": C, "chi": chi, "mH": mE - hr * mM, "hmax": hmax,
            "d_T": hmax / Tc ** 2, "d_h": N / Tc + 0 * hr,
            "d_TT": varH / Tc ** 4 + 2 * hmax / Tc ** 3,
            "d_Th": (np.sqrt(varH * varM) / Tc + N) / Tc ** 2,
            "d_hh": varM / Tc ** 2}
