"""Benchmark: exact enumeration of the +-J 8x5 square torus on one MI355X.

One step = the whole hot path on one synthetic input:
  1. ising_enumerate: g(E, M) over all 2^40 configurations of the 8x5 torus
     with couplings +-1 (seeded) (zero-fill + the Gray-walk/LDS-histogram
     kernel),
  2. ising_moments: log Z, <E>, <M>, C, chi on the 256 x 8 (T, h) grid in FP64.
value = configurations enumerated per second (2^40 per step / step time).

Beside it (same line): the 6x6 J = 1 torus (2^36), the halved form, the
256-lattice batch, the autograd backward, and the oracle on the host cores.

Prints ONE JSON line on stdout (diagnostics go to stderr).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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
INT_ALU_TARGET = 0.5

# Sources of the enumeration kernel: the hardware-counter figures below hold
# only for the build they were taken on; if the sources' hash differs, they
# are reported as null.
KERNEL_SOURCES = ['paper_1110_2561_amd/csrc/enumerate.hip', 'paper_1110_2561_amd/csrc/walk.h',
                  'paper_1110_2561_amd/csrc/plan.cpp', 'paper_1110_2561_amd/csrc/internal.h']
KERNEL_SHA256 = "0ee52cfb0a44b48835888db5caab1e85a40135e04ba9ead95b4bbbae0ddae7d1"

# rocprofv3 counters of k_enumerate per workload, per launch (profiles/k_enumerate_*):
#   hbm_bytes: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (KiB -> bytes), the factors being
#              what a 512 MiB copy kernel reads on the same counters;
#   int32_valu: SQ_INSTS_VALU_INT32 x 64 lanes / configurations;
#   valu: SQ_INSTS_VALU x 64 lanes / configurations.
COUNTERS = {
    "torus8x5_pm": {
        "kernel": "k_enumerate<8, 2>",
        "hbm_bytes": int((92.0 * 2.0 + 1257.21875 * 1.0) * 1024),
        "int32_valu": 18194651285 * 64 / 2 ** 40,
        "valu": 19681281869 * 64 / 2 ** 40,
    },
    "torus6x6": {
        "kernel": "k_enumerate<8, 1>",
        "hbm_bytes": int((85.0 * 2.0 + 936.28125 * 1.0) * 1024),
        "int32_valu": 1133076202 * 64 / 2 ** 36,
        "valu": 1210787418 * 64 / 2 ** 36,
    },
}

def sources_sha256() -> str:
    """SHA-256 over the library's C/HIP sources and header (provenance of the
    measured build; the line may be produced where no git history exists)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    files = sorted(glob.glob(os.path.join(_ROOT, "paper_1110_2561_amd", "csrc", "*"))) + \
        [os.path.join(_ROOT, "include", "ising.h")]
    for f in files:
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def counters_valid(workload: str) -> bool:
    import hashlib
    if workload not in COUNTERS:
        return False
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(_ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest() == KERNEL_SHA256


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(lat, sample_log2: int) -> dict:
    """The oracle, as it stands, on the host cores, on the first 2^sample_log2
    configurations of the same lattice.  For a square torus with couplings
    +-1 that is the oracle's version of the paper's own scheme (Section 3:
    one bit word per row, satisfied bonds by XOR, NOT, mask and popcount, with
    one more XOR against a per-row sign mask for J = -1 bonds); its brute force
    over bonds, which any lattice takes, is timed beside it on a smaller
    sample."""
    from oracle import native
    from paper_1110_2561_amd import lattice as L
    threads = native.default_threads()
    host = f"{_cpu_model()}; {os.cpu_count()} logical CPUs visible, {threads} threads used"
    row_scheme = (lat.kind == "square_torus" and set(int(v) for v in lat.bond_J) <= {-1, 1}
                  and min(lat.dims) >= 3)
    bf_log2 = sample_log2 - 2 if row_scheme else sample_log2
    count = 1 << bf_log2
    t0 = time.perf_counter()
    native.count_range(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J, 0, count, threads)
    bf_dt = time.perf_counter() - t0
    bf = {"value": count / bf_dt, "sample": f"configurations [0, 2^{bf_log2}), {bf_dt:.1f} s wall"}
    if not row_scheme:
        return {"value": bf["value"], "unit": "configs/s", "cores": threads, "kind": "oracle",
                "sample": f"configurations [0, 2^{bf_log2}) of the {lat.n_spins}-spin workload, "
                          f"brute force over bonds, {bf_dt:.1f} s wall", "host": host}
    Lx, Ly = lat.dims
    Jh, Jv = L.torus_coupling_grids(lat)
    count = 1 << sample_log2
    t0 = time.perf_counter()
    native.row_words(Lx, Ly, 0, count, threads, Jh, Jv)
    dt = time.perf_counter() - t0
    return {"value": count / dt, "unit": "configs/s", "cores": threads, "kind": "oracle",
            "sample": f"configurations [0, 2^{sample_log2}) of the {lat.n_spins}-spin workload, "
                      f"the paper's row bit-word scheme (XOR/NOT/mask/popcount, per-row sign masks "
                      f"for J = -1), {dt:.1f} s wall",
            "bruteforce": bf, "host": host}


def gray_step_ops(lat) -> int:
    """Integer ops of one popcount-based Gray step (a flip, then per coupling
    class an AND + popcount-accumulate and a scale by J_c, then the sign and
    the E/M update, then the bin update), for masks held in one 32-bit word
    with a good site ordering: 1 + 2 n_c + n_c + 2 + 1."""
    n_c = len({int(v) for v in lat.bond_J if int(v) != 0}) or 1
    return 1 + 2 * n_c + n_c + 2 + 1


def copy_calibration(nbytes: int) -> int:
    """A plain copy kernel of known size: it reads and writes nbytes once per
    launch, which calibrates the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = nbytes // 8
    src = torch.arange(n, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copied {n * 8} bytes x 3")
    return 0


def _median_ms(fn, reps: int) -> float:
    """Median event-timed duration of fn() on the current stream, in ms."""
    import numpy as np
    import torch
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        ts.append(a.elapsed_time(b))
    return float(np.median(ts))


def bench_batched(plain_rate: float, reps: int) -> dict:
    """The 256-lattice batch in one persistent launch, and the captured graph
    of {zero, enumerate, moments}; reported beside the plain kernel."""
    import torch

    from dataclasses import asdict

    from paper_1110_2561_amd import api, autotune
    from paper_1110_2561_amd import lattice as L
    w = L.workload("batch256")
    # chunk / tile / copy choices picked by the autotuner on this GPU (timed
    # outside the measurement; not cached, so the line reflects this run)
    t0 = time.perf_counter()
    tune, tried = autotune.autotune_batch(w["lattices"], reps=2, use_cache=False)
    tune_s = time.perf_counter() - t0
    plan = api.BatchPlan(w["lattices"], tune)
    g = plan.new_tables()
    api.batch_enumerate(plan, out=g)
    torch.cuda.synchronize()
    g_host = g.cpu()
    for i, lat in enumerate(plan.lattices):   # every table sums to 2^N
        assert int(plan.table(g_host, i).view(torch.int64).sum()) == 1 << lat.n_spins
    total = plan.total_configs
    ms = _median_ms(lambda: api.batch_enumerate(plan, out=g), reps)
    # halved: each member over its configurations with the top spin up, mirrored
    g2 = plan.new_tables()
    api.batch_enumerate(plan, out=g2, symmetric=True)
    torch.cuda.synchronize()
    assert torch.equal(g2.cpu(), g_host), "halved batch differs from the full batch"
    hms = _median_ms(lambda: api.batch_enumerate(plan, out=g2, symmetric=True), reps)
    graph = api.BatchGraph(plan, w["T"], w["h"])
    graph.replay()
    torch.cuda.synchronize()
    gms = _median_ms(graph.replay, reps)
    hgraph = api.BatchGraph(plan, w["T"], w["h"], symmetric=True)
    hgraph.replay()
    torch.cuda.synchronize()
    assert torch.equal(hgraph.g_all.cpu(), g_host), "halved graph differs from the full batch"
    hgms = _median_ms(hgraph.replay, reps)
    kinds = sorted({lat.kind for lat in plan.lattices})
    return {
        "workload": f"batch256: {len(plan)} lattices ({', '.join(kinds)}), N in "
                    f"[{int(plan.n_spins.min())}, {int(plan.n_spins.max())}], J in {{-2,-1,1,2}}, one persistent launch",
        "configs": total,
        "value": total / (ms * 1e-3),
        "unit": "configs/s",
        "enumerate_ms": ms,
        "graph_ms": gms,
        "graph": f"zero + batched enumerate + batched moments on {len(w['T'])} T x {len(w['h'])} h",
        "vs_plain": total / (ms * 1e-3) / plain_rate,
        "halved_ms": hms,
        "halved_graph_ms": hgms,
        "halved_covered": total / (hms * 1e-3),
        "halved": "each member over its configurations with the top spin up, then g(E,M) += g(E,-M); "
                  "checked bit-identical to the full batch",
        "tune": {k: v for k, v in asdict(tune).items() if v},
        "autotune": f"{len(tried)} candidate tunes timed in {tune_s:.1f} s",
    }


def bench_symmetric(plan, g, configs: int, plain_rate: float, reps: int) -> dict:
    """The same table from half the configurations (global spin flip,
    g(E, M) = g(E, -M)); configurations covered vs enumerated reported apart."""
    import torch

    from paper_1110_2561_amd import api
    ref = g.clone()
    api.enumerate_symmetric(plan, out=g)
    torch.cuda.synchronize()
    assert torch.equal(g, ref), "halved table differs from the full enumeration"
    ms = _median_ms(lambda: api.enumerate_symmetric(plan, out=g), reps)
    return {
        "method": "enumerate the configurations with the top prefix spin up, then g(E,M) += g(E,-M)",
        "ms": ms,
        "configs_covered_per_s": configs / (ms * 1e-3),
        "configs_enumerated_per_s": configs / 2 / (ms * 1e-3),
        "vs_plain": configs / (ms * 1e-3) / plain_rate,
    }


def bench_other_lattice(name: str, reps: int) -> dict:
    """k_enumerate on another single-lattice workload, timed like the main
    kernel (median of event-timed launches), with its LDS-atomic fraction."""
    import numpy as np
    import torch
    from paper_1110_2561_amd import api
    from paper_1110_2561_amd import lattice as L

    lat = L.workload(name)["lattice"]
    plan = api.Plan(lat)
    g = plan.new_table()
    api.enumerate_g(plan, out=g)      # warm-up (device copy of the plan)
    torch.cuda.synchronize()
    ms = _median_ms(lambda: api.enumerate_g(plan, out=g), reps)
    gh = g.cpu().numpy()
    assert int(gh.sum(dtype=np.uint64)) == 1 << lat.n_spins and np.array_equal(gh, gh[:, ::-1])
    rate = (1 << lat.n_spins) / (ms * 1e-3)
    out = {
        "lattice": f"{lat.kind} {lat.describe()['dims']} (N={lat.n_spins}, {lat.n_bonds} bonds, "
                   + ("J=1)" if set(int(v) for v in lat.bond_J) == {1} else f"seeded +-J, seed {lat.seed})"),
        "kernel_ms": ms,
        "value": rate,
        "unit": "configs/s",
        "lds_atomic_frac": rate / LDS_ATOMIC_PEAK,
        "check": "sum g = 2^N and g(E, M) = g(E, -M)",
    }
    if counters_valid(name):
        c = COUNTERS[name]
        out["int32_valu_per_config"] = c["int32_valu"]
        out["int_alu_frac"] = c["int32_valu"] * rate / INT_VALU_PEAK
    return out


def bench_autograd(plain_rate: float, reps: int) -> dict:
    """log Z(T, h, J) on the 64 x 64 grid with its hand-written backward
    (dT, dh from g; per-bond dJ by recomputed enumeration): the time of
    torch.autograd.grad through the autograd Function, and of the library's
    one-call backward (ising_logz_backward) that the Function issues."""
    import torch

    from paper_1110_2561_amd import api
    from paper_1110_2561_amd import autograd as ag
    from paper_1110_2561_amd import lattice as L
    w = L.workload("autograd")
    out = {"grid": [len(w["T"]), len(w["h"])], "dtype": "f64 sums over u32/u64 enumeration",
           "backward": "dT, dh from g; per-bond dJ by a recomputed walk over all 2^N configurations",
           "backward_ms": "torch.autograd.grad(sum log Z, (T, h, J)) through the autograd Function, "
                          "with PyTorch's engine overhead",
           "library_backward_ms": "the same gradients from one ising_logz_backward call (all its kernels on "
                                  "one stream, no host synchronisation)",
           "backward_symmetric": "the same, dJ walking the half with the top spin up with weights "
                                 "W(E,M) + W(E,-M) (spin-flip symmetry); checked equal to the full form",
           "lattices": []}
    for lat in w["lattices"]:
        f = ag.IsingLogZ(lat)
        T = torch.as_tensor(w["T"], dtype=torch.float64, device="cuda").requires_grad_(True)
        h = torch.as_tensor(w["h"], dtype=torch.float64, device="cuda").requires_grad_(True)
        J = f.couplings()
        res = {}

        def fwd():
            res["lz"] = f(T, h, J)

        def bwd():
            res["g"] = torch.autograd.grad(res["lz"].sum(), (T, h, J), retain_graph=True)

        fwd()
        bwd()
        torch.cuda.synchronize()
        # sum rule: sum_b J_b d(sum log Z)/dJ_b = -sum_{T,h} <E>/T
        m = api.moments(f.g, f.plan.e_min, lat.n_spins, T.detach(), h.detach())
        lhs = float((J.detach() * res["g"][2]).sum())
        rhs = float((-m["mean_E"] / T.detach()[:, None]).sum())
        assert abs(lhs - rhs) <= 1e-9 * max(1.0, abs(rhs)), (lhs, rhs)
        fms = _median_ms(fwd, reps)
        bms = _median_ms(bwd, reps)
        lz, G = res["lz"].detach(), torch.ones_like(res["lz"])
        Td, hd = T.detach(), h.detach()

        def lib():
            res["lib"] = api.logz_backward(f.plan, f.g, Td, hd, lz, G)

        lib()
        torch.cuda.synchronize()
        assert all(torch.equal(a, b) for a, b in zip(res["lib"], res["g"])), "library backward differs"
        lms = _median_ms(lib, reps)
        f.symmetric_backward = True          # the per-bond sums over half the configurations
        g_full = res["g"]
        bwd()
        torch.cuda.synchronize()
        for a, b in zip(g_full, res["g"]):
            assert torch.allclose(a, b, rtol=1e-10, atol=1e-12 * float(a.abs().max())), "halved backward differs"
        sms = _median_ms(bwd, reps)
        f.symmetric_backward = False
        configs = 1 << lat.n_spins
        out["lattices"].append({
            "lattice": f"{lat.kind} {lat.describe()['dims']} (N={lat.n_spins}, {lat.n_bonds} bonds, "
                       + ("J=1)" if set(int(v) for v in lat.bond_J) == {1} else f"seeded +-J, seed {lat.seed})"),
            "forward_ms": fms,
            "backward_ms": bms,
            "library_backward_ms": lms,
            "backward_value": configs / (lms * 1e-3),
            "unit": "configs/s",
            "vs_plain": configs / (lms * 1e-3) / plain_rate,
            "backward_symmetric_ms": sms,
            "backward_symmetric_covered": configs / (sms * 1e-3),
            "symmetric_vs_plain": configs / (sms * 1e-3) / plain_rate,
        })
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="torus8x5_pm", choices=["torus8x5_pm", "torus6x6", "torus4x4"])
    ap.add_argument("--cpu-sample-log2", type=int, default=33)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tile-bits", type=int, default=0, help="plan tile width (0 = the plan's choice)")
    ap.add_argument("--inner-bits", type=int, default=0, help="plan chunk width (0 = the plan's choice)")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and autograd measurements")
    ap.add_argument("--only", choices=["halving", "batched", "autograd", "6x6"], default=None,
                    help="of the measurements beside the headline, run only this one (for profiling)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="BYTES",
                    help="only run a plain device-to-device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
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
    tuned = bool(args.tile_bits or args.inner_bits)
    plan = api.Plan(lat, api.Tune(inner_bits=args.inner_bits, tile_bits=args.tile_bits) if tuned else None)
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

    valid = counters_valid(args.workload) and not tuned
    cnt = COUNTERS.get(args.workload, {}) if valid else {}
    int32_per_config = cnt.get("int32_valu")
    int_frac = int32_per_config * achieved / INT_VALU_PEAK if valid else None
    ops = gray_step_ops(lat)
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
                        f"{lat.kind} (N={lat.n_spins}, {lat.n_bonds} bonds, "
                        + ("J=1" if set(int(v) for v in lat.bond_J) == {1} else f"J=+-1 from seed {lat.seed}")
                        + f"), then FP64 log Z and moments on {len(T)} T x {len(h)} h",
            "n_spins": lat.n_spins,
            "configs_per_step": configs,
            "grid": [len(T), len(h)],
            "thermo_dtype": "f64",
            "table_dtype": "u64",
        },
        "roofline": {
            "bound": "alu",
            "ceiling": "the LDS atomic unit: one ds_add_u32 per configuration, 16 lanes/clk/CU "
                       "(256 CU x 16 x 2.4 GHz)",
            "achieved": achieved / 1e12,
            "peak": LDS_ATOMIC_PEAK / 1e12,
            "unit": "T increments/s",
            "frac": achieved / LDS_ATOMIC_PEAK,
            "traffic": cnt.get("hbm_bytes") if valid else None,
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": f"{cnt.get('kernel', 'k_enumerate')} (event-timed on its stream, with its zero-fill)",
            "kernel_ms": kern_ms,
        },
        "int_alu": {
            "achieved": int32_per_config * achieved / 1e12 if valid else None,
            "peak": INT_VALU_PEAK / 1e12,
            "unit": "Tops/s",
            "frac": int_frac,
            "target_frac": INT_ALU_TARGET,
            "target_met": (int_frac >= INT_ALU_TARGET) if valid else None,
            "int32_valu_per_config": int32_per_config,
            "basis": "rocprofv3 SQ_INSTS_VALU_INT32 x 64 lanes per configuration, times the event-timed rate",
            "why_below_target": "every configuration needs one LDS atomic, and the LDS atomic unit "
                                "(16 lanes/clk/CU) binds the walk at about one int32 op per configuration, "
                                "a quarter of the int32 VALU issue rate (64 lanes/clk/CU); narrower tiles "
                                "do more integer work per configuration and run slower",
            "op_equivalent": {
                "ops_per_config": ops,
                "rate": ops * achieved / 1e12,
                "unit": "T int-op equivalents/s",
                "ratio_to_int32_peak": ops * achieved / INT_VALU_PEAK,
                "note": "not a fraction of peak: the rate a popcount-based Gray step (flip; AND, "
                        "popcount-accumulate and J scale per coupling class; sign; E/M update; bin update) "
                        "would need to match this throughput; the kernel executes int32_valu_per_config",
            },
        },
    }
    line["build"] = {"sources_sha256": sources_sha256(), "arch": torch.cuda.get_device_properties(0).gcnArchName,
                     "cus": torch.cuda.get_device_properties(0).multi_processor_count}
    if not args.no_extras:
        def want(name):
            return args.only is None or args.only == name
        if want("halving"):
            line["z2_halving"] = bench_symmetric(plan, g, configs, achieved, reps=5)
        if want("batched"):
            line["batched"] = bench_batched(achieved, reps=5)
        if want("autograd"):
            line["autograd"] = bench_autograd(achieved, reps=5)
        if want("6x6") and args.workload != "torus6x6":
            line["enumeration_6x6"] = bench_other_lattice("torus6x6", reps=10)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(lat, args.cpu_sample_log2)
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
