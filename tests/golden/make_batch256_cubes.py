"""Write the oracle's degeneracy tables of the batch256 workload's 3x3x3 cubes.

    python tests/golden/make_batch256_cubes.py      # -> tests/golden/batch256_cubes.npz

The batch256 workload mixes square tori, free-boundary triangular patches and
simple-cubic 3x3x3 tori with couplings in {-2, -1, 1, 2}.  The tori and the
patches have fast exact oracle counts (transfer matrix, banded count); the
cubes (2^27 configurations, 81 bonds) take the brute force over every
configuration and bond, the definition of g(E, M) after Eq. (2) of
Peretyatko et al. (Section 2), about 4 s each on 8 host threads.  This script
runs that brute force (oracle.native.count_all, nothing else) once per cube
and stores the tables, so the GPU tests can compare every member exactly.

Stored (numpy .npz, no pickles):
  member     int32 [C]     index of the cube in the batch256 list
  seed       uint64 [C]    the member's coupling seed (identity check)
  bonds_sha  S64 [C]       SHA-256 of the member's bond list (i, j, J as int32)
  n_e        int32 [C]     table rows (2S + 1); columns are n_up = 0 .. 27
  offsets    int64 [C + 1] entries of cube c: [offsets[c], offsets[c+1])
  e_idx      int16 [.]     row E + S of a nonzero bin
  n_up       int8 [.]      column of the bin
  count      uint32 [.]    g(E, M) of the bin (< 2^27)
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

_ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if _ROOT not in sys.path:
    sys.path.insert(0, _ROOT)

from oracle import native                       # noqa: E402
from paper_1110_2561_amd import lattice as L    # noqa: E402  (inputs only)

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch256_cubes.npz")


def bonds_sha(lat) -> bytes:
    h = hashlib.sha256()
    for a in (lat.bond_i, lat.bond_j, lat.bond_J):
        h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    return h.hexdigest().encode()


def cube_members(lats):
    return [i for i, lat in enumerate(lats) if lat.kind == "cubic_torus"]


def main() -> int:
    lats = L.workload("batch256")["lattices"]
    members = cube_members(lats)
    seeds, shas, n_e, offsets, e_idx, n_up, count = [], [], [], [0], [], [], []
    t0 = time.perf_counter()
    for k, i in enumerate(members):
        lat = lats[i]
        g = native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
        assert int(g.sum()) == 1 << lat.n_spins and int(g.max()) < 1 << 32
        e, n = np.nonzero(g)
        seeds.append(lat.seed)
        shas.append(bonds_sha(lat))
        n_e.append(g.shape[0])
        e_idx.append(e.astype(np.int16))
        n_up.append(n.astype(np.int8))
        count.append(g[e, n].astype(np.uint32))
        offsets.append(offsets[-1] + e.size)
        print(f"cube {k + 1}/{len(members)} (member {i}): {e.size} nonzero bins, "
              f"{time.perf_counter() - t0:.0f} s", flush=True)
    np.savez_compressed(OUT, member=np.array(members, np.int32), seed=np.array(seeds, np.uint64),
                        bonds_sha=np.array(shas, dtype="S64"), n_e=np.array(n_e, np.int32),
                        offsets=np.array(offsets, np.int64), e_idx=np.concatenate(e_idx),
                        n_up=np.concatenate(n_up), count=np.concatenate(count))
    print(f"wrote {OUT}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
