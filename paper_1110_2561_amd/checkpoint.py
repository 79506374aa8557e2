"""Resumable enumeration: a plan's chunk range in pieces, with an atomic
checkpoint (partial table, next chunk) written after every piece.

Chunk ranges are additive (ising_enumerate_range adds the counts of a range
to a table), so a run that stops anywhere - a crash, a killed job, a time
limit - resumes from its last checkpoint and ends with exactly the table of
an uninterrupted run: the piece in flight when it stopped is simply redone.
This is the single-GPU form of the paper's split of the loops into
independent parts whose counts are summed at the end (Section 3d).

Chunk numbering depends on the plan (spin order, chunk width), so a
checkpoint carries a fingerprint of the lattice and the plan's layout, and a
run refuses a checkpoint made for a different one.

    from paper_1110_2561_amd import api, checkpoint
    g, finished = checkpoint.run(api.Plan(lat), "run.ckpt.npz")
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np
import torch

__all__ = ["fingerprint", "load", "save", "run"]


def fingerprint(plan) -> str:
    """SHA-256 of the lattice (bonds in input order) and the plan's layout
    (spin order, chunk and tile width, chunk count, table shape)."""
    lat = plan.lattice
    h = hashlib.sha256()
    h.update(json.dumps({"n_spins": int(lat.n_spins), "inner_bits": int(plan.inner_bits),
                         "tile_bits": int(plan.tile_bits), "n_chunks": int(plan.n_chunks),
                         "table": [int(plan.n_e), int(plan.n_m), int(plan.e_min)]}).encode())
    for a in (lat.bond_i, lat.bond_j, lat.bond_J, plan.bit_of_site):
        h.update(np.ascontiguousarray(a, dtype=np.int64).tobytes())
    return h.hexdigest()


def save(path: str, plan, table: np.ndarray, next_chunk: int) -> None:
    """Write the checkpoint atomically: a temporary file, then a rename, so a
    stop during the write leaves the previous checkpoint intact."""
    table = np.ascontiguousarray(table, dtype=np.uint64)
    if table.shape != (plan.n_e, plan.n_m):
        raise ValueError(f"table shape {table.shape}, plan table {(plan.n_e, plan.n_m)}")
    if not 0 <= int(next_chunk) <= plan.n_chunks:
        raise ValueError(f"next chunk {next_chunk} outside [0, {plan.n_chunks}]")
    tmp = path + ".tmp"
    with open(tmp, "wb") as f:
        np.savez(f, table=table.view(np.int64), next_chunk=np.array(int(next_chunk), dtype=np.uint64),
                 n_chunks=np.array(int(plan.n_chunks), dtype=np.uint64),
                 fingerprint=np.array(fingerprint(plan)))
        f.flush()
        os.fsync(f.fileno())
    os.replace(tmp, path)


def load(path: str, plan):
    """(table, next_chunk) of the checkpoint at path, or None if there is none.
    Raises ValueError if it was made for another lattice or plan layout."""
    if not os.path.exists(path):
        return None
    with np.load(path, allow_pickle=False) as z:
        fp = str(z["fingerprint"])
        table = z["table"].view(np.uint64).copy()
        next_chunk = int(z["next_chunk"])
        n_chunks = int(z["n_chunks"])
    if fp != fingerprint(plan) or n_chunks != plan.n_chunks:
        raise ValueError(f"checkpoint {path} belongs to another lattice or plan layout")
    if table.shape != (plan.n_e, plan.n_m) or not 0 <= next_chunk <= n_chunks:
        raise ValueError(f"checkpoint {path} is malformed")
    return table, next_chunk


def run(plan, path: str, piece_chunks: int | None = None, max_pieces: int | None = None,
        range_fn=None, device: str = "cuda"):
    """Enumerate all of plan's chunks, resuming from the checkpoint at path if
    there is one, in pieces of piece_chunks chunks (default: 1/16 of the
    range), checkpointing after each.  Stops early after max_pieces pieces.

    Returns (g, finished): the table so far (uint64 [n_e][n_m] on device) and
    whether every chunk is counted.  range_fn(first_chunk, n_chunks, g) adds a
    range's counts to g; it defaults to api.enumerate_range on the GPU.
    """
    if range_fn is None:
        from . import api

        def range_fn(first, n, g):
            api.enumerate_range(plan, first, n, g)
    state = load(path, plan)
    host, nxt = state if state is not None else (np.zeros((plan.n_e, plan.n_m), dtype=np.uint64), 0)
    g = torch.from_numpy(host.view(np.int64)).view(torch.uint64).to(device)
    step = max(1, plan.n_chunks // 16) if piece_chunks is None else int(piece_chunks)
    if step < 1:
        raise ValueError("piece_chunks must be >= 1")
    pieces = 0
    while nxt < plan.n_chunks and (max_pieces is None or pieces < max_pieces):
        n = min(step, plan.n_chunks - nxt)
        range_fn(nxt, n, g)
        nxt += n
        pieces += 1
        save(path, plan, g.cpu().numpy(), nxt)   # the copy waits for the piece
    return g, nxt == plan.n_chunks
