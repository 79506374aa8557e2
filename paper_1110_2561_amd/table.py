"""The degeneracy table as the paper's program reports it: one row
(count, M, E) per nonzero bin.

In the paper the root process collects the counts, sorts them and saves them
(Section 3d), and Section 4 Table 1 prints them as (Nc, M, E).  Here rows are
sorted by M, then E, both ascending; M = 2 n_up - N is the spin excess and E
the exchange energy.  Host-side formatting only: the table itself comes from
the library (api.enumerate_g and friends).
"""
from __future__ import annotations

from typing import Iterable

import numpy as np

__all__ = ["rows", "write", "read"]


def _host(g) -> np.ndarray:
    if hasattr(g, "detach"):          # a torch tensor (uint64, any device)
        import torch
        g = g.detach().cpu().view(torch.int64).numpy().view(np.uint64)
    g = np.asarray(g)
    if g.ndim != 2:
        raise ValueError("g must be a 2-D [n_e][n_m] table")
    return g.astype(np.uint64, copy=False)


def rows(g, e_min: int, n_spins: int) -> list[tuple[int, int, int]]:
    """(count, M, E) of every nonzero bin of the dense table g[E - e_min][n_up],
    sorted by M and then E."""
    g = _host(g)
    if g.shape[1] != n_spins + 1:
        raise ValueError(f"table has {g.shape[1]} n_up columns, expected {n_spins + 1}")
    e_idx, n_up = np.nonzero(g)
    out = [(int(g[e, u]), 2 * int(u) - n_spins, int(e) + e_min) for e, u in zip(e_idx, n_up)]
    out.sort(key=lambda r: (r[1], r[2]))
    return out


def write(dest, g, e_min: int, n_spins: int, header: Iterable[str] = ()) -> None:
    """Write the rows as text, one 'count M E' line per bin, after '#' header
    lines; dest is a path or a text file object."""
    lines = [f"# {h}" for h in header] + ["# count M E"]
    lines += [f"{c} {m} {e}" for c, m, e in rows(g, e_min, n_spins)]
    text = "\n".join(lines) + "\n"
    if isinstance(dest, (str, bytes)) or hasattr(dest, "__fspath__"):
        with open(dest, "w") as f:
            f.write(text)
    else:
        dest.write(text)


def read(src) -> list[tuple[int, int, int]]:
    """The rows of a file written by write (comment lines skipped)."""
    f = open(src) if isinstance(src, (str, bytes)) or hasattr(src, "__fspath__") else src
    try:
        out = []
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                c, m, e = (int(v) for v in line.split())
                out.append((c, m, e))
        return out
    finally:
        if f is not src:
            f.close()
