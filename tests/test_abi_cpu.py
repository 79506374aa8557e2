"""The C-ABI library without a GPU: it loads, exports every declared symbol,
validates its inputs and builds plans (plan creation makes no HIP call)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1110_2561_amd import lattice as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1110_2561_amd import _lib
    return _lib


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "ising.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ising_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    syms = _declared_symbols()
    assert {"ising_plan_create", "ising_enumerate", "ising_enumerate_range", "ising_logz", "ising_moments"} <= set(syms)
    for s in syms:
        assert hasattr(lib.lib, s), s


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.ising_version()
    for code, name in lib.STATUS.items():
        assert lib.ising_status_str(code).decode() == name


def _create(lib, n, bi, bj, bJ, tune=None):
    bi = np.asarray(bi, dtype=np.int32); bj = np.asarray(bj, dtype=np.int32); bJ = np.asarray(bJ, dtype=np.int32)
    p = lib.i32p
    lat = lib.ising_lattice(n, bi.shape[0], bi.ctypes.data_as(p), bj.ctypes.data_as(p), bJ.ctypes.data_as(p))
    h = ctypes.c_void_p()
    rc = lib.ising_plan_create(ctypes.byref(lat), ctypes.byref(tune) if tune else None, ctypes.byref(h))
    if rc == 0:
        lib.ising_plan_destroy(h)
    return rc, lib.ising_last_error().decode()


@pytest.mark.parametrize("n,bi,bj,bJ,code", [
    (0, [], [], [], -2),
    (65, [], [], [], -2),
    (4, [0], [0], [1], -3),           # self-bond
    (4, [0], [4], [1], -3),           # endpoint out of range
    (4, [-1], [2], [1], -3),
    (4, [0], [1], [1 << 21], -4),     # |J| too large
    (4, [0, 1, 2], [1, 2, 3], [1 << 20, 1 << 20, 1], -4),   # sum |J| too large
    (9, list(range(8)) + [0], list(range(1, 9)) + [2], [1, 2, 3, 4, 5, 6, 7, 8, 9], -7),  # 9 coupling classes
])
def test_plan_create_rejects_bad_input(lib, n, bi, bj, bJ, code):
    rc, msg = _create(lib, n, bi, bj, bJ)
    assert rc == code and msg.startswith(lib.STATUS[code])


def test_plan_create_rejects_bad_tune(lib):
    lat = L.square_torus(3, 3)
    for tune in (lib.ising_tune(0, 9, 0, 0, 0), lib.ising_tune(0, 0, 17, 0, 0), lib.ising_tune(0, 0, 0, 3, 0),
                 lib.ising_tune(26, 0, 0, 0, 0), lib.ising_tune(2, 4, 0, 0, 0)):
        rc, _ = _create(lib, lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J, tune)
        assert rc == -1


def test_null_arguments(lib):
    assert lib.ising_plan_create(None, None, None) == -1
    assert lib.ising_hist_shape(None, None, None, None) == -1
    assert lib.ising_enumerate(None, None, None) == -1
    assert lib.ising_plan_destroy(None) == 0


def test_large_histogram_is_rejected(lib):
    # A star of large, incommensurate couplings: its compact energy range
    # needs far more bins than the LDS holds.
    n = 40
    bi = [0] * (n - 1)
    bj = list(range(1, n))
    bJ = [3 ** (k % 8) + 1000 * (k // 8) for k in range(n - 1)]
    rc, msg = _create(lib, n, bi, bj, bJ)
    assert rc in (-4, -7), msg


def _plan(lat, **tune):
    from paper_1110_2561_amd.api import Plan, Tune
    return Plan(lat, Tune(**tune) if tune else None)


@pytest.mark.parametrize("lat,S", [(L.square_torus(4, 4), 32), (L.square_torus(6, 6), 72),
                                   (L.workload("torus8x5_pm")["lattice"], 80), (L.cubic_torus(3), 81)])
def test_plan_shape_and_layout(lat, S):
    p = _plan(lat)
    assert (p.n_e, p.n_m, p.e_min) == (2 * S + 1, lat.n_spins + 1, -S)
    assert sorted(p.bit_of_site.tolist()) == list(range(lat.n_spins))
    assert p.n_chunks == 1 << (lat.n_spins - p.inner_bits)
    assert 1 <= p.tile_bits <= p.inner_bits <= lat.n_spins
    # tile sites are pairwise uncoupled
    tile = set(np.nonzero(p.bit_of_site < p.tile_bits)[0].tolist())
    for i, j in zip(lat.bond_i, lat.bond_j):
        assert not (i in tile and j in tile)


def test_plan_tune_is_honoured():
    p = _plan(L.square_torus(6, 6), inner_bits=14, tile_bits=3)
    assert (p.inner_bits, p.tile_bits, p.n_chunks) == (14, 3, 1 << 22)


def test_tiny_systems_plan():
    for lat in (L.Lattice(1, [], [], []), L.Lattice(2, [0], [1], [-1]), L.Lattice(3, [], [], [])):
        p = _plan(lat)
        assert p.inner_bits <= lat.n_spins and p.n_chunks >= 1


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1110_2561_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, flags=re.M), f
                assert "liboracle" not in src, f


def test_batch_plan_layout_on_cpu():
    from paper_1110_2561_amd.api import BatchPlan, Tune
    lats = [L.square_torus(4, 4), L.ring(7), L.cubic_torus(3, L.choice_couplings(81, 1)), L.Lattice(1, [], [], [])]
    b = BatchPlan(lats, Tune(prefix_bits=10))
    sizes = [(2 * l.abs_coupling_sum + 1) * (l.n_spins + 1) for l in lats]
    assert b.offsets.tolist() == [0] + np.cumsum(sizes).tolist()
    assert b.n_spins.tolist() == [16, 7, 27, 1]
    assert b.total_configs == sum(1 << l.n_spins for l in lats)


def test_batch_plan_errors_name_the_member():
    from paper_1110_2561_amd.api import BatchPlan, IsingError
    with pytest.raises(IsingError):
        BatchPlan([])
    with pytest.raises(IsingError, match="member 1"):
        BatchPlan([L.ring(5), L.Lattice(3, [0], [0], [1])])
    with pytest.raises(IsingError, match="65535"):
        BatchPlan([L.ring(3)] * 65536)


def test_wrappers_reject_tables_a_kernel_cannot_read():
    # host, non-contiguous, wrongly typed or shaped tensors are refused in
    # Python, before any pointer reaches the library
    import torch

    from paper_1110_2561_amd import api
    from paper_1110_2561_amd import lattice as L
    g_host = torch.zeros((33, 17), dtype=torch.uint64)
    for fn in (api.log_z, api.moments, api.logz_derivatives):
        with pytest.raises(ValueError):
            fn(g_host, -32, 16, [1.0], [0.0])
    with pytest.raises(ValueError):
        api.bin_weights(g_host, -32, 16, [1.0], [0.0], torch.zeros((1, 1), dtype=torch.float64),
                        torch.zeros((1, 1), dtype=torch.float64))
    plan = api.Plan(L.square_torus(4, 4))
    with pytest.raises(ValueError):
        api.bond_backward(plan, torch.zeros((plan.n_e, plan.n_m), dtype=torch.float64))
    with pytest.raises(ValueError):
        api.enumerate_g(plan, out=torch.zeros((plan.n_e, plan.n_m), dtype=torch.uint64))


def test_autotune_cache_key_names_the_batch_and_the_build():
    from paper_1110_2561_amd import autotune
    a = [L.square_torus(4, 4), L.ring(9)]
    b = [L.square_torus(4, 4), L.ring(10)]
    ka, kb = autotune.batch_key(a), autotune.batch_key(b)
    assert ka == autotune.batch_key(list(a)) and ka != kb
    assert ka.split(":")[1] == autotune._library_tag()


def test_bench_refuses_more_than_one_gpu():
    # the library has no multi-GPU path; bench.py says so and exits non-zero
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2 and "one GPU" in r.stderr and r.stdout == ""
