"""Benchmark: exact enumeration of the 6x6 square torus on one MI355X.

One step = the whole hot path on one synthetic input:
  1. ising_enumerate: g(E, M) over all 2^36 configurations (zero-fill +
     the Gray-walk/LDS-histogram kernel),
  2. ising_moments: log Z, <E>, <M>, C, chi on the 256 x 8 (T, h) grid in FP64.
value = configurations enumerated per second (2^36 per step / step time).

Prints ONE JSON line on stdout (diagnostics go to stderr).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

_ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, _ROOT)

METRIC = "spin configs enumerated/sec (1 GPU) + % int-ALU peak; batched & autograd vs plain"
# Roofline of the enumeration kernel: one LDS atomic increment (ds_add_u32)
# per configuration.  The LDS serves 128 B/clk/CU of bank accesses; an atomic
# read-modify-write of 4 B costs two, so 16 atomic lanes/clk/CU:
# 256 CU x 16 x 2.4 GHz.
LDS_ATOMIC_PEAK = 256 * 16 * 2.4e9
# Integer VALU: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz (non-packed 32-bit ops).
INT_VALU_PEAK = 256 * 64 * 2.4e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(lat, sample_log2: int) -> dict:
    """The oracle's brute force, as it stands, on the first 2^sample_log2
    configurations of the same lattice, on the host cores."""
    from oracle import native
    threads = native.default_threads()
    count = 1 << sample_log2
    t0 = time.perf_counter()
    native.count_range(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J, 0, count, threads)
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "configs/s", "cores": threads, "kind": "oracle",
            "sample": f"configurations [0, 2^{sample_log2}) of the {lat.n_spins}-spin workload, "
                      f"brute force over bonds, {dt:.1f} s wall"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="torus6x6", choices=["torus6x6", "torus8x5_pm", "torus4x4"])
    ap.add_argument("--cpu-sample-log2", type=int, default=31)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(sharding would split the chunk range per GPU and sum the uint64 tables); "
              "run with --gpus 1", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_1110_2561_amd import api
    from paper_1110_2561_amd import lattice as L

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    w = L.workload(args.workload)
    lat, T, h = w["lattice"], w["T"], w["h"]
    plan = api.Plan(lat)
    configs = 1 << lat.n_spins
    g = plan.new_table()
    Tt = torch.as_tensor(T, dtype=torch.float64, device="cuda")
    ht = torch.as_tensor(h, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    log(f"workload {args.workload}: N={lat.n_spins} B={lat.n_bonds} chunks={plan.n_chunks} "
        f"inner_bits={plan.inner_bits} tile_bits={plan.tile_bits} table={plan.n_e}x{plan.n_m}")

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        api.enumerate_g(plan, out=g)
        if ev is not None:
            ev[1].record(stream)
        return api.moments(g, plan.e_min, lat.n_spins, Tt, ht)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        out = step(events[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in events]))
    ms_per_step = dt * 1e3 / args.steps
    value = configs * args.steps / dt
    achieved = configs / (kern_ms * 1e-3)
    g_host = g.cpu().numpy()
    assert int(g_host.sum(dtype=np.uint64)) == configs % (1 << 64), "table does not sum to 2^N"
    log(f"enumerate launch {kern_ms:.3f} ms avg, step {ms_per_step:.3f} ms, "
        f"log Z finite: {bool(torch.isfinite(out['log_z']).all())}")

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "configs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: exhaustive g(E,M) of the {lat.describe()['dims']} "
                        f"{lat.kind} (N={lat.n_spins}, {lat.n_bonds} bonds), then FP64 log Z and "
                        f"moments on {len(T)} T x {len(h)} h",
            "n_spins": lat.n_spins,
            "configs_per_step": configs,
            "grid": [len(T), len(h)],
            "thermo_dtype": "f64",
            "table_dtype": "u64",
        },
        "roofline": {
            "bound": "alu",
            "op": "LDS atomic increment (ds_add_u32), one per configuration",
            "achieved": achieved / 1e12,
            "peak": LDS_ATOMIC_PEAK / 1e12,
            "unit": "Tops/s",
            "frac": achieved / LDS_ATOMIC_PEAK,
            "traffic": None,
            "kernel": "k_enumerate (event-timed with its zero-fill)",
            "kernel_ms": kern_ms,
        },
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lat, args.cpu_sample_log2)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
