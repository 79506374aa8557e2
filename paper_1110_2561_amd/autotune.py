"""Autotuner for the enumeration's decomposition knobs.

The plan's defaults (8-bit tile, ~4 tasks per block) are near the LDS
atomic ceiling for one large lattice.  A batch mixes lattices of different
size, coordination and coupling spread, where chunk size (prefix_bits), tile
width and histogram copies trade per-task set-up against load balance.  The
tuner times a small grid of candidates with the real kernel on the current
GPU and caches the winner in a JSON file keyed by the GPU architecture and a
hash of the batch's lattices.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from dataclasses import asdict

import numpy as np
import torch

from . import api
from .lattice import Lattice

DEFAULT_CANDIDATES = [
    api.Tune(),                       # batch default: members with 2^14-configuration chunks
    api.Tune(inner_bits=12),
    api.Tune(inner_bits=16),
    api.Tune(inner_bits=18),
    api.Tune(prefix_bits=18),
    api.Tune(inner_bits=14, replicas=8),
    api.Tune(inner_bits=14, tile_bits=7),
]


def cache_path() -> str:
    return os.environ.get("ISING_AUTOTUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "paper_1110_2561_amd", "autotune.json")


def _library_tag() -> str:
    """Hash of the loaded library file: a rebuilt kernel invalidates cached choices."""
    from . import _lib
    h = hashlib.sha256()
    with open(_lib.LIB_PATH, "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:12]


def batch_key(lattices) -> str:
    h = hashlib.sha256()
    for lat in lattices:
        h.update(np.int64(lat.n_spins).tobytes())
        for a in (lat.bond_i, lat.bond_j, lat.bond_J):
            h.update(np.ascontiguousarray(a, dtype=np.int32).tobytes())
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] if torch.cuda.is_available() else "cpu"
    return f"{arch}:{_library_tag()}:{h.hexdigest()[:24]}"


def _time_batch(plan: api.BatchPlan, reps: int) -> float:
    g = plan.new_tables()
    api.batch_enumerate(plan, out=g)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        api.batch_enumerate(plan, out=g)
        b.record()
        torch.cuda.synchronize()
        best = min(best, a.elapsed_time(b))
    return best


def autotune_batch(lattices: list[Lattice], candidates=None, reps: int = 2, use_cache: bool = True,
                   verbose: bool = False) -> tuple[api.Tune, dict]:
    """Fastest Tune for this batch on this GPU, and the timings (ms) seen."""
    key = batch_key(lattices)
    path = cache_path()
    cache = {}
    if use_cache and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if use_cache and key in cache:
        return api.Tune(**cache[key]["tune"]), cache[key]["timings"]
    timings = {}
    best, best_ms = None, float("inf")
    t0 = time.perf_counter()
    for cand in candidates or DEFAULT_CANDIDATES:
        try:
            plan = api.BatchPlan(lattices, cand)
        except api.IsingError:
            continue
        ms = _time_batch(plan, reps)
        plan.close()
        timings[json.dumps(asdict(cand), sort_keys=True)] = ms
        if verbose:
            print(f"autotune {asdict(cand)}: {ms:.3f} ms", flush=True)
        if ms < best_ms:
            best, best_ms = cand, ms
    if best is None:
        raise RuntimeError("no candidate tune is valid for this batch")
    if use_cache:
        cache[key] = {"tune": asdict(best), "timings": timings, "seconds": time.perf_counter() - t0}
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return best, timings
