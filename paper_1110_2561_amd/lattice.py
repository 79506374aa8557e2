"""Seeded synthetic inputs: finite Ising lattices as integer bond lists.

This module builds inputs only.  It holds none of the counting or
thermodynamic arithmetic of the method; both the library and its test oracle
receive the plain arrays it produces (site count, bond endpoints, integer
couplings).

The paper's Hamiltonian (Section 2, Eq. (1)) sums J_ij S_i S_j over the
nearest neighbours of every site with a factor 1/2, so each bond contributes
once: E = -sum_b J_b s_i s_j.  A lattice is therefore a multiset of bonds
(i, j, J) with integer J.  The paper treats the 2D square lattice with
periodic boundaries (Z = 4) and names 3D lattices and sign-changing couplings
as generalisations (Section 2, Section 3); the builders below cover the
square torus, the 1D ring, a free-boundary triangular patch, the simple-cubic
torus and seeded competing couplings.

Canonical bond order: sites ascending by index, and for each site its bonds
in the +x, +y, (+z | +diagonal) directions.  Couplings drawn from a seed are
assigned in this order.

A torus side of length 2 produces two distinct bonds between the same pair of
sites (i -> i+1 and i+1 -> i wrap); both are kept, which matches the Z-fold
neighbour sum of Eq. (1).  Side length 1 would produce self-bonds and is
rejected.
"""
from __future__ import annotations

import dataclasses
from typing import Iterable, Sequence

import numpy as np

__all__ = [
    "Lattice",
    "SplitMix64",
    "square_torus",
    "ring",
    "triangular_free",
    "cubic_torus",
    "pm_couplings",
    "choice_couplings",
    "random_bond_lattice",
    "torus_coupling_grids",
    "workload",
    "T_GRID",
]

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """Vigna's SplitMix64 generator (public-domain reference definition).

    state += 0x9E3779B97F4A7C15; z = state;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB;
    return z ^ (z >> 31)             (all arithmetic modulo 2^64)
    """

    def __init__(self, seed: int):
        self.state = int(seed) & _MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)


@dataclasses.dataclass(frozen=True)
class Lattice:
    """A finite Ising system: N spins and a multiset of integer-coupled bonds."""

    n_spins: int
    bond_i: np.ndarray  # int32 [B]
    bond_j: np.ndarray  # int32 [B]
    bond_J: np.ndarray  # int32 [B]
    kind: str = "custom"
    dims: tuple = ()
    seed: int | None = None

    def __post_init__(self):
        for name in ("bond_i", "bond_j", "bond_J"):
            a = np.ascontiguousarray(np.asarray(getattr(self, name), dtype=np.int32))
            object.__setattr__(self, name, a)
        if not (self.bond_i.shape == self.bond_j.shape == self.bond_J.shape):
            raise ValueError("bond arrays must have equal length")

    @property
    def n_bonds(self) -> int:
        return int(self.bond_i.shape[0])

    @property
    def abs_coupling_sum(self) -> int:
        """S = sum_b |J_b|; every configuration has E in [-S, S]."""
        return int(np.abs(self.bond_J.astype(np.int64)).sum())

    def relabel(self, new_index_of_site: Sequence[int]) -> "Lattice":
        """The same system with site u renamed new_index_of_site[u]."""
        p = np.asarray(new_index_of_site, dtype=np.int64)
        if sorted(p.tolist()) != list(range(self.n_spins)):
            raise ValueError("relabelling must be a permutation of the sites")
        return Lattice(self.n_spins, p[self.bond_i], p[self.bond_j], self.bond_J.copy(),
                       kind=self.kind, dims=self.dims, seed=self.seed)

    def describe(self) -> dict:
        return {"kind": self.kind, "dims": list(self.dims), "n_spins": self.n_spins,
                "n_bonds": self.n_bonds, "seed": self.seed}

    def to_json(self) -> str:
        """A self-contained JSON descriptor: the bond list with its couplings
        (bonds as [i, j, J] in input order) and the builder's description."""
        import json
        d = self.describe()
        d["bonds"] = [[int(i), int(j), int(J)] for i, j, J in zip(self.bond_i, self.bond_j, self.bond_J)]
        return json.dumps(d)

    @staticmethod
    def from_json(text: str) -> "Lattice":
        """The lattice of a descriptor written by to_json (bond order kept)."""
        import json
        d = json.loads(text)
        b = np.asarray(d.get("bonds", []), dtype=np.int64).reshape(-1, 3)
        if b.shape[0] != int(d.get("n_bonds", b.shape[0])):
            raise ValueError("descriptor's n_bonds does not match its bond list")
        if np.abs(b).max(initial=0) >= 2 ** 31:
            raise ValueError("bond endpoints and couplings must fit int32")
        return Lattice(int(d["n_spins"]), b[:, 0], b[:, 1], b[:, 2], kind=str(d.get("kind", "custom")),
                       dims=tuple(int(x) for x in d.get("dims", ())), seed=d.get("seed"))


def _couplings(n: int, J) -> np.ndarray:
    if np.isscalar(J):
        return np.full(n, int(J), dtype=np.int32)
    a = np.asarray(J, dtype=np.int32).reshape(-1)
    if a.shape[0] != n:
        raise ValueError(f"expected {n} couplings, got {a.shape[0]}")
    return a


def square_torus(Lx: int, Ly: int, J=1, seed: int | None = None) -> Lattice:
    """Lx x Ly square lattice with periodic boundaries (Z = 4), 2*Lx*Ly bonds.

    Site (x, y) has index y*Lx + x.  Bond order per site: +x then +y.
    """
    if Lx < 2 or Ly < 2:
        raise ValueError("torus sides must be >= 2")
    bi, bj = [], []
    for y in range(Ly):
        for x in range(Lx):
            u = y * Lx + x
            bi.append(u); bj.append(y * Lx + (x + 1) % Lx)
            bi.append(u); bj.append(((y + 1) % Ly) * Lx + x)
    return Lattice(Lx * Ly, bi, bj, _couplings(len(bi), J), kind="square_torus",
                   dims=(Lx, Ly), seed=seed)


def ring(N: int, J=1, seed: int | None = None) -> Lattice:
    """1D periodic chain of N >= 3 spins (Ising's 1D case, Z = 2)."""
    if N < 3:
        raise ValueError("ring needs N >= 3")
    bi = list(range(N))
    bj = [(u + 1) % N for u in range(N)]
    return Lattice(N, bi, bj, _couplings(N, J), kind="ring", dims=(N,), seed=seed)


def triangular_free(N: int, Lx: int, J=1, seed: int | None = None) -> Lattice:
    """Triangular patch with free boundaries: rows of Lx sites filled row-major
    to exactly N sites (the last row may be partial); bonds +x, +y and the
    +(1, 1) diagonal wherever both ends exist (interior Z = 6)."""
    if N < 1 or Lx < 1:
        raise ValueError("bad triangular patch")
    bi, bj = [], []

    def idx(x, y):
        u = y * Lx + x
        return u if (0 <= x < Lx and u < N) else None

    for u in range(N):
        x, y = u % Lx, u // Lx
        for dx, dy in ((1, 0), (0, 1), (1, 1)):
            v = idx(x + dx, y + dy)
            if v is not None:
                bi.append(u); bj.append(v)
    return Lattice(N, bi, bj, _couplings(len(bi), J), kind="triangular_free",
                   dims=(Lx, N), seed=seed)


def cubic_torus(L: int = 3, J=1, seed: int | None = None) -> Lattice:
    """L x L x L simple-cubic lattice with periodic boundaries (Z = 6).

    Site (x, y, z) has index (z*L + y)*L + x; bonds +x, +y, +z per site.
    """
    if L < 2:
        raise ValueError("cubic side must be >= 2")
    bi, bj = [], []
    for z in range(L):
        for y in range(L):
            for x in range(L):
                u = (z * L + y) * L + x
                bi.append(u); bj.append((z * L + y) * L + (x + 1) % L)
                bi.append(u); bj.append((z * L + (y + 1) % L) * L + x)
                bi.append(u); bj.append((((z + 1) % L) * L + y) * L + x)
    return Lattice(L ** 3, bi, bj, _couplings(len(bi), J), kind="cubic_torus",
                   dims=(L, L, L), seed=seed)


def pm_couplings(n: int, seed: int) -> np.ndarray:
    """n couplings in {-1, +1}, +1 iff the top bit of a SplitMix64 draw is set
    (P(+1) = 1/2), drawn in canonical bond order."""
    rng = SplitMix64(seed)
    return np.array([1 if (rng.next() >> 63) else -1 for _ in range(n)], dtype=np.int32)


def choice_couplings(n: int, seed: int, values: Iterable[int] = (-2, -1, 1, 2)) -> np.ndarray:
    """n couplings drawn uniformly from `values` (length a power of two) using
    the top bits of SplitMix64 draws."""
    vals = list(values)
    bits = len(vals).bit_length() - 1
    if 1 << bits != len(vals):
        raise ValueError("number of coupling values must be a power of two")
    rng = SplitMix64(seed)
    if bits == 0:
        return np.full(n, vals[0], dtype=np.int32)
    return np.array([vals[rng.next() >> (64 - bits)] for _ in range(n)], dtype=np.int32)


def random_bond_lattice(N: int, n_bonds: int, seed: int, values=(-2, -1, 1, 2)) -> Lattice:
    """Random multigraph on N sites (no self-bonds) with couplings from `values`."""
    rng = SplitMix64(seed)
    bi, bj = [], []
    while len(bi) < n_bonds and N >= 2:
        i = rng.next() % N
        j = rng.next() % N
        if i != j:
            bi.append(i); bj.append(j)
    J = choice_couplings(len(bi), seed ^ 0x5EED, values)
    return Lattice(N, bi, bj, J, kind="random", dims=(N, n_bonds), seed=seed)


def torus_coupling_grids(lat: Lattice):
    """(Jh, Jv) grids [Ly][Lx] of a square_torus lattice in canonical order:
    Jh[y][x] couples (x, y)-(x+1, y), Jv[y][x] couples (x, y)-(x, y+1)."""
    if lat.kind != "square_torus":
        raise ValueError("not a square torus")
    Lx, Ly = lat.dims
    J = lat.bond_J.reshape(Ly, Lx, 2)
    return np.ascontiguousarray(J[:, :, 0]), np.ascontiguousarray(J[:, :, 1])


# Temperature grid shared by the workloads: T in [0.5, 5].
def T_GRID(n: int) -> np.ndarray:
    return np.linspace(0.5, 5.0, n)


_PM_SEED_8x5 = 20111025
_PM_SEED_CUBE = 27
_BATCH_SEED = 1110_2561


def workload(name: str) -> dict:
    """The synthetic workloads of the benchmark and the parity tests.

    Returns a dict with the lattice(s) and the (T, h) grids.
    """
    if name == "torus4x4":
        return {"lattice": square_torus(4, 4), "T": T_GRID(64), "h": np.array([0.0, 0.1, 0.5])}
    if name == "torus6x6":
        return {"lattice": square_torus(6, 6), "T": T_GRID(256),
                "h": np.array([0.0, 0.01, 0.05, 0.1, 0.25, 0.5, 1.0, 2.0])}
    if name == "torus8x5_pm":
        J = pm_couplings(80, _PM_SEED_8x5)
        return {"lattice": square_torus(8, 5, J, seed=_PM_SEED_8x5), "T": T_GRID(256),
                "h": np.array([0.0, 0.01, 0.05, 0.1, 0.25, 0.5, 1.0, 2.0])}
    if name == "batch256":
        return {"lattices": batch_lattices(256, _BATCH_SEED), "T": T_GRID(64),
                "h": np.array([0.0, 0.1, 0.5])}
    if name == "autograd":
        return {"lattices": [square_torus(6, 6), cubic_torus(3),
                             cubic_torus(3, pm_couplings(81, _PM_SEED_CUBE), seed=_PM_SEED_CUBE)],
                "T": T_GRID(64), "h": np.linspace(-1.0, 1.0, 64)}
    raise KeyError(name)


def _torus_shapes():
    """(Lx, Ly) with 3 <= Lx <= Ly and 16 <= Lx*Ly <= 32."""
    return [(a, b) for a in range(3, 33) for b in range(a, 33) if 16 <= a * b <= 32]


def batch_lattices(n: int, seed: int) -> list:
    """Mixed batch: instance t is a square torus (t % 3 == 0), a free-boundary
    triangular patch (t % 3 == 1) or the 3x3x3 cubic torus (t % 3 == 2);
    sizes N in [16, 32] and couplings uniform in {-2, -1, 1, 2}, all drawn
    from SplitMix64 streams derived from `seed`."""
    rng = SplitMix64(seed)
    shapes = _torus_shapes()
    out = []
    for t in range(n):
        s = rng.next()
        kind = t % 3
        if kind == 0:
            Lx, Ly = shapes[rng.next() % len(shapes)]
            base = square_torus(Lx, Ly)
        elif kind == 1:
            N = 16 + rng.next() % 17
            Lx = 4 + rng.next() % 3
            base = triangular_free(N, Lx)
        else:
            base = cubic_torus(3)
        J = choice_couplings(base.n_bonds, s)
        out.append(Lattice(base.n_spins, base.bond_i, base.bond_j, J, kind=base.kind,
                           dims=base.dims, seed=s))
    return out
