"""Command line: enumerate one lattice on the GPU and write its degeneracy
table (count, M, E per nonzero bin), optionally with log Z and moments.

    python -m paper_1110_2561_amd torus:6x6 --table g.txt --T 0.5:5:64 --h 0,0.1
    python -m paper_1110_2561_amd torus:8x5 --pm 20111025 --symmetric
    python -m paper_1110_2561_amd lattice.json --checkpoint run.npz

Lattices: torus:LxxLy, ring:N, cubic:L, triangular:NxLx (N spins in rows of
Lx), or a JSON descriptor (lattice.Lattice.to_json).  --pm SEED replaces the
couplings by seeded +-1 draws, --couplings SEED:v1,v2,... by seeded draws
from the given values.  Thermodynamics go to stdout (or --thermo FILE) as
JSON: log Z, <E>, <M>, C and chi on the T x h grid.
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import lattice as L


def parse_lattice(spec: str) -> L.Lattice:
    """A lattice from a builder spec or a JSON descriptor file."""
    kind, _, arg = spec.partition(":")
    try:
        if kind == "torus":
            lx, ly = (int(v) for v in arg.lower().split("x"))
            return L.square_torus(lx, ly)
        if kind == "ring":
            return L.ring(int(arg))
        if kind == "cubic":
            return L.cubic_torus(int(arg))
        if kind == "triangular":
            n, lx = (int(v) for v in arg.lower().split("x"))
            return L.triangular_free(n, lx)
    except ValueError as e:
        raise SystemExit(f"bad lattice spec {spec!r}: {e}")
    with open(spec) as f:
        return L.Lattice.from_json(f.read())


def with_couplings(lat: L.Lattice, pm: int | None, couplings: str | None) -> L.Lattice:
    if pm is not None:
        J = L.pm_couplings(lat.n_bonds, pm)
        seed = pm
    elif couplings:
        s, _, vals = couplings.partition(":")
        seed = int(s)
        J = L.choice_couplings(lat.n_bonds, seed, tuple(int(v) for v in vals.split(",")))
    else:
        return lat
    return L.Lattice(lat.n_spins, lat.bond_i, lat.bond_j, J, kind=lat.kind, dims=lat.dims, seed=seed)


def parse_grid(text: str) -> np.ndarray:
    """'a:b:n' (n points from a to b) or a comma-separated list."""
    if ":" in text:
        a, b, n = text.split(":")
        return np.linspace(float(a), float(b), int(n))
    return np.array([float(v) for v in text.split(",")])


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(prog="python -m paper_1110_2561_amd", description=__doc__.split("\n\n")[0])
    ap.add_argument("lattice", help="torus:6x6 | ring:N | cubic:L | triangular:NxLx | FILE.json")
    ap.add_argument("--pm", type=int, default=None, metavar="SEED", help="seeded +-1 couplings")
    ap.add_argument("--couplings", default=None, metavar="SEED:V1,V2,...", help="seeded couplings from a value set")
    ap.add_argument("--table", default=None, help="write the table here (default: no table output)")
    ap.add_argument("--T", default=None, help="temperatures, a:b:n or a list")
    ap.add_argument("--h", default="0", help="fields, a:b:n or a list (default 0)")
    ap.add_argument("--thermo", default=None, help="write the thermodynamics JSON here (default stdout)")
    ap.add_argument("--symmetric", action="store_true", help="enumerate half and mirror M -> -M")
    ap.add_argument("--checkpoint", default=None, help="resumable run with this checkpoint file")
    args = ap.parse_args(argv)

    import torch
    from . import api, checkpoint, table

    if not torch.cuda.is_available():
        print("no GPU visible: the enumeration runs only on the GPU", file=sys.stderr)
        return 2
    lat = with_couplings(parse_lattice(args.lattice), args.pm, args.couplings)
    plan = api.Plan(lat)
    if args.checkpoint:
        g, done = checkpoint.run(plan, args.checkpoint)
        assert done
    elif args.symmetric:
        g = api.enumerate_symmetric(plan)
    else:
        g = api.enumerate_g(plan)
    torch.cuda.synchronize()
    total = int(g.cpu().view(torch.int64).numpy().view(np.uint64).sum(dtype=np.uint64))
    if total != (1 << lat.n_spins) % (1 << 64):
        print(f"table sums to {total}, not 2^{lat.n_spins}", file=sys.stderr)
        return 1
    desc = lat.describe()
    if args.table:
        table.write(args.table, g, plan.e_min, lat.n_spins,
                    header=[f"{desc['kind']} {desc['dims']} N={lat.n_spins} bonds={lat.n_bonds} seed={desc['seed']}",
                            f"sum of counts = 2^{lat.n_spins}"])
    if args.T is not None:
        T, h = parse_grid(args.T), parse_grid(args.h)
        m = api.moments(g, plan.e_min, lat.n_spins, T, h)
        out = {"lattice": desc, "T": T.tolist(), "h": h.tolist(),
               **{k: v.cpu().numpy().tolist() for k, v in m.items()}}
        text = json.dumps(out)
        if args.thermo:
            with open(args.thermo, "w") as f:
                f.write(text + "\n")
        else:
            print(text)
    return 0


if __name__ == "__main__":
    sys.exit(main())
