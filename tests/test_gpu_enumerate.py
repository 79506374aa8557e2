"""Parity of the HIP enumeration (through the C ABI) with the CPU oracle.

Integer results must be bit-exact.  Small systems are compared with the
brute-force definition, the full-size tori with the transfer-matrix count,
and sampled chunk ranges at full size with the brute force over exactly the
same configurations.
"""
import numpy as np
import pytest
import torch

from conftest import load_table1, nonzero_bins
from oracle import closed_forms, native
from paper_1110_2561_amd import lattice as L

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1110_2561_amd import api as A
    return A


def _gpu_g(api, lat, tune=None):
    plan = api.Plan(lat, api.Tune(**tune) if tune else None)
    g = api.enumerate_g(plan)
    torch.cuda.synchronize()
    return plan, g.cpu().numpy()


def _bf(lat):
    return native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)


def _tm(lat):
    return native.tm_torus(*L.torus_coupling_grids(lat))


def test_table1_4x4(api):
    lat = L.square_torus(4, 4)
    _, g = _gpu_g(api, lat)
    assert nonzero_bins(g, -32, 16) == load_table1()
    np.testing.assert_array_equal(g, _bf(lat))


def _tri(N, Lx, seed):
    base = L.triangular_free(N, Lx)
    return L.triangular_free(N, Lx, L.choice_couplings(base.n_bonds, seed))


SMALL = [
    (L.Lattice(1, [], [], []), None),
    (L.Lattice(2, [0], [1], [-3]), None),
    (L.Lattice(5, [], [], []), None),                                   # no bonds
    (L.ring(3), None),
    (L.ring(7, L.pm_couplings(7, 2)), {"inner_bits": 4, "tile_bits": 1}),
    (L.square_torus(2, 2), None),                                        # doubled bonds
    (L.square_torus(3, 3, L.choice_couplings(18, 7)), None),
    (L.square_torus(3, 4, L.pm_couplings(24, 11)), {"inner_bits": 8, "tile_bits": 3}),
    (L.square_torus(4, 4), {"inner_bits": 16, "tile_bits": 6}),          # one chunk
    (L.square_torus(4, 4), {"inner_bits": 6, "tile_bits": 6, "replicas": 1}),
    (L.square_torus(4, 5, L.choice_couplings(40, 3)), {"tile_bits": 5, "waves_per_block": 3}),
    (L.square_torus(4, 5), {"tile_bits": 2, "max_blocks": 1}),
    (_tri(11, 4, 3), None),
    (_tri(19, 5, 8), {"replicas": 2}),
    (L.random_bond_lattice(9, 20, 5), None),                             # repeated pairs
    (L.random_bond_lattice(13, 30, 6, values=(-3, 1)), {"tile_bits": 4}),
    (L.random_bond_lattice(17, 60, 7), {"waves_per_block": 1, "replicas": 4}),
    (L.random_bond_lattice(22, 45, 8, values=(-2, -1, 1, 2)), None),
    (L.cubic_torus(2), None),
    (L.Lattice(12, list(range(11)), list(range(1, 12)), [1] * 11), {"tile_bits": 6}),  # open chain
]


@pytest.mark.parametrize("lat,tune", SMALL, ids=[f"{l.kind}{l.n_spins}-{i}" for i, (l, _) in enumerate(SMALL)])
def test_small_systems_bit_exact(api, lat, tune):
    print(f"case {lat.kind} N={lat.n_spins} B={lat.n_bonds} tune={tune}", flush=True)
    _, g = _gpu_g(api, lat, tune)
    np.testing.assert_array_equal(g, _bf(lat))


def test_every_tile_width_6x4(api):
    lat = L.square_torus(6, 4, L.pm_couplings(48, 21))
    ref = _tm(lat)
    for tb in range(1, 7):
        for kb in (tb, tb + 3, 12):
            print(f"tile_bits={tb} inner_bits={kb}", flush=True)
            _, g = _gpu_g(api, lat, {"tile_bits": tb, "inner_bits": kb})
            np.testing.assert_array_equal(g, ref)


def test_torus6x6_full(api):
    lat = L.workload("torus6x6")["lattice"]
    _, g = _gpu_g(api, lat)
    np.testing.assert_array_equal(g, _tm(lat))


def test_torus8x5_pm_full(api):
    lat = L.workload("torus8x5_pm")["lattice"]
    _, g = _gpu_g(api, lat)
    ref = _tm(lat)
    assert int(ref.max()) > 1 << 32
    np.testing.assert_array_equal(g, ref)


def test_periodic_flush_path(api):
    # One replica and 2^21-configuration chunks: every counter may take 2^31
    # adds per task, so the block flushes after every task.
    lat = L.square_torus(8, 4, L.pm_couplings(64, 5))
    _, g = _gpu_g(api, lat, {"inner_bits": 21, "replicas": 1, "max_blocks": 1})
    np.testing.assert_array_equal(g, _tm(lat))


def test_run_to_run_identical(api):
    lat = L.workload("torus8x5_pm")["lattice"]
    plan = api.Plan(lat)
    a = api.enumerate_g(plan).cpu()
    b = api.enumerate_g(plan).cpu()
    assert torch.equal(a, b)


def test_ranges_sum_to_whole(api):
    lat = L.workload("torus6x6")["lattice"]
    plan = api.Plan(lat)
    whole = api.enumerate_g(plan)
    parts = torch.zeros_like(whole)
    C = plan.n_chunks
    cuts = [0, 1, 1000, C // 3 + 7, C - 5, C]
    for a, b in zip(cuts[:-1], cuts[1:]):
        api.enumerate_range(plan, a, b - a, parts)
    torch.cuda.synchronize()
    assert torch.equal(whole.cpu(), parts.cpu())


def test_checkpoint_and_resume(api, tmp_path):
    """An interrupted run resumes from a saved partial table and chunk offset:
    a first plan enumerates a prefix of the chunk range and checkpoints
    (table, next chunk) to disk; a fresh plan loads it and finishes."""
    lat = L.workload("torus8x5_pm")["lattice"]
    whole = api.enumerate_g(api.Plan(lat)).cpu().numpy()
    plan1 = api.Plan(lat)
    g = torch.zeros((plan1.n_e, plan1.n_m), dtype=torch.uint64, device="cuda")
    stop = plan1.n_chunks // 3 + 11
    step = max(1, stop // 4)
    done = 0
    while done < stop:                       # the first run, in pieces
        n = min(step, stop - done)
        api.enumerate_range(plan1, done, n, g)
        done += n
    torch.cuda.synchronize()
    np.save(tmp_path / "partial.npy", g.cpu().numpy().view(np.int64))
    (tmp_path / "next_chunk.txt").write_text(str(done))
    del g, plan1                             # the run ends here
    plan2 = api.Plan(lat)
    resumed = torch.from_numpy(np.load(tmp_path / "partial.npy")).view(torch.uint64).cuda()
    nxt = int((tmp_path / "next_chunk.txt").read_text())
    api.enumerate_range(plan2, nxt, plan2.n_chunks - nxt, resumed)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(resumed.cpu().numpy(), whole)


@pytest.mark.parametrize("which", [1, 2], ids=["cubic3", "cubic3_pm"])
def test_autograd_workload_cubes_bit_exact(api, which):
    """The autograd workload's 3x3x3 cubes (J = 1 and seeded +-J, 2^27
    configurations each), plain and halved, against the brute force."""
    lat = L.workload("autograd")["lattices"][which]
    assert lat.kind == "cubic_torus" and lat.n_spins == 27
    ref = native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    plan = api.Plan(lat)
    np.testing.assert_array_equal(api.enumerate_g(plan).cpu().numpy(), ref)
    np.testing.assert_array_equal(api.enumerate_symmetric(plan).cpu().numpy(), ref)


def test_checkpoint_runner_resumes(api, tmp_path):
    """The library's checkpointed runner on the GPU: stopped after two pieces,
    resumed by a fresh plan, equal to the transfer-matrix table (8x5 +-J)."""
    from paper_1110_2561_amd import checkpoint
    lat = L.workload("torus8x5_pm")["lattice"]
    path = str(tmp_path / "run.npz")
    g, done = checkpoint.run(api.Plan(lat), path, max_pieces=2)
    assert not done
    g, done = checkpoint.run(api.Plan(lat), path)
    assert done
    np.testing.assert_array_equal(g.cpu().numpy(), native.tm_torus(*L.torus_coupling_grids(lat)))


LARGE = {
    "torus6x6": L.workload("torus6x6")["lattice"],
    "torus8x5_pm": L.workload("torus8x5_pm")["lattice"],
    "torus8x8_pm": L.square_torus(8, 8, L.pm_couplings(128, 64)),                      # N = 64, 8 copies
    "random50": L.random_bond_lattice(50, 120, 50, values=(-2, -1, 1, 2)),           # 4 copies
    "cubic4": L.cubic_torus(4, L.choice_couplings(192, 4)),                           # N = 64, 6 neighbours
}


@pytest.mark.parametrize("name", list(LARGE))
def test_sampled_range_vs_bruteforce(api, name):
    """Full-size plan, a sampled chunk range: the same configurations counted
    by the brute force after renaming sites to the plan's bit positions."""
    lat = LARGE[name]
    plan = api.Plan(lat)
    print(f"{name}: N={lat.n_spins} inner={plan.inner_bits} tile={plan.tile_bits} chunks={plan.n_chunks}", flush=True)
    k = plan.inner_bits
    n_ch = max(1, (1 << 26) >> k)
    rng = np.random.default_rng(1234)
    first = int(rng.integers(0, plan.n_chunks - n_ch))
    g = torch.zeros((plan.n_e, plan.n_m), dtype=torch.uint64, device="cuda")
    api.enumerate_range(plan, first, n_ch, g)
    torch.cuda.synchronize()
    rel = lat.relabel(plan.bit_of_site)
    ref = native.count_range(rel.n_spins, rel.bond_i, rel.bond_j, rel.bond_J, first << k, n_ch << k)
    np.testing.assert_array_equal(g.cpu().numpy(), ref)


def test_range_errors(api):
    plan = api.Plan(L.square_torus(4, 4))
    g = plan.new_table()
    with pytest.raises(api.IsingError):
        api.enumerate_range(plan, plan.n_chunks, 1, g)
    with pytest.raises(api.IsingError):
        api.enumerate_range(plan, 0, plan.n_chunks + 1, g)
    api.enumerate_range(plan, plan.n_chunks, 0, g)    # empty range is fine


def test_side_stream(api):
    lat = L.square_torus(4, 5, L.choice_couplings(40, 3))
    plan = api.Plan(lat)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        g = api.enumerate_g(plan, stream=s)
    s.synchronize()
    np.testing.assert_array_equal(g.cpu().numpy(), _bf(lat))


# --------------------------------------------------------------------------
# spin-flip halving: half the configurations, mirrored M -> -M
# --------------------------------------------------------------------------

@pytest.mark.parametrize("lat,tune", SMALL, ids=[f"{l.kind}{l.n_spins}-{i}" for i, (l, _) in enumerate(SMALL)])
def test_symmetric_small_systems_bit_exact(api, lat, tune):
    print(f"symmetric case {lat.kind} N={lat.n_spins} tune={tune}", flush=True)
    plan = api.Plan(lat, api.Tune(**tune) if tune else None)
    g = plan.new_table()
    g.fill_(12345)                                          # stale contents must be overwritten
    api.enumerate_symmetric(plan, out=g)
    np.testing.assert_array_equal(g.cpu().numpy(), _bf(lat))


@pytest.mark.parametrize("name", ["torus6x6", "torus8x5_pm"])
def test_symmetric_full_size_matches_transfer_matrix(api, name):
    lat = L.workload(name)["lattice"]
    plan = api.Plan(lat)
    g = api.enumerate_symmetric(plan).cpu().numpy()
    np.testing.assert_array_equal(g, _tm(lat))


def _sweep_cases(n_cases=60, seed=20240611):
    """Seeded random multigraphs (N 2-20, up to 3N bonds, 1-8 coupling values,
    some pairs repeated) with a random tune each."""
    rng = L.SplitMix64(seed)
    values = [(-1, 1), (-2, -1, 1, 2), (1,), (-3, 2), (-2, 2, 3, -5), (-1, 1, 2, -2, 3, -3, 4, -4)]
    tunes = [None, {"tile_bits": 1}, {"tile_bits": 3}, {"inner_bits": 6}, {"replicas": 2},
             {"waves_per_block": 2}, {"max_blocks": 2}, {"tile_bits": 2, "replicas": 8}, {"prefix_bits": 3}]
    out = []
    for k in range(n_cases):
        n = 2 + rng.next() % 19
        nb = rng.next() % (3 * n + 1)
        lat = L.random_bond_lattice(n, nb, rng.next() & 0xFFFFFFFF, values=values[rng.next() % len(values)])
        out.append((lat, tunes[rng.next() % len(tunes)]))
    return out


@pytest.mark.parametrize("k", range(60))
def test_seeded_random_sweep(api, k):
    """Each case: the full, halved and range-split enumerations bit-exact against
    the brute force, and the per-bond backward (full and halved) against the
    oracle's split counts."""
    lat, tune = _sweep_cases()[k]
    print(f"case {k}: N={lat.n_spins} bonds={lat.n_bonds} tune={tune}", flush=True)
    ref = native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    try:
        plan = api.Plan(lat, api.Tune(**tune) if tune else None)
    except api.IsingError:                         # a tune this lattice cannot take
        try:
            plan = api.Plan(lat)
        except api.IsingError as e:                # more than 8 merged couplings: refused cleanly
            assert e.code == -7 and "merged couplings" in str(e), e
            return
    np.testing.assert_array_equal(api.enumerate_g(plan).cpu().numpy(), ref)
    np.testing.assert_array_equal(api.enumerate_symmetric(plan).cpu().numpy(), ref)
    g = torch.zeros((plan.n_e, plan.n_m), dtype=torch.uint64, device="cuda")
    cut = plan.n_chunks // 3
    api.enumerate_range(plan, cut, plan.n_chunks - cut, g)
    api.enumerate_range(plan, 0, cut, g)
    np.testing.assert_array_equal(g.cpu().numpy(), ref)
    if lat.n_bonds:
        from oracle import grad
        g2, gp = native.bond_split(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
        W = np.where(g2 > 0, np.random.default_rng(k).standard_normal(g2.shape), 0.0)
        refJ = grad.bond_grad_from_weights(g2, gp, W)
        scale = (np.abs(W) * g2.astype(np.float64)).sum()
        for sym in (False, True):
            dJ = api.bond_backward(plan, torch.from_numpy(W).cuda(), symmetric=sym).cpu().numpy()
            np.testing.assert_allclose(dJ, refJ, rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("k", range(12))
def test_property_sweep_21_to_30_spins(api, k):
    """Seeded random multigraphs of 21-30 spins (brute force is too slow here):
    sum g = 2^N, binomial marginals, g(E, M) = g(E, -M), and the halved and
    range-split tables equal to the full one."""
    rng = L.SplitMix64(777 + k)
    n = 21 + rng.next() % 10
    lat = L.random_bond_lattice(n, n + rng.next() % (2 * n), rng.next() & 0xFFFFFFFF,
                                values=[(-1, 1), (-2, -1, 1, 2), (1,), (-3, 2)][k % 4])
    plan = api.Plan(lat)
    print(f"case {k}: N={n} bonds={lat.n_bonds} chunks={plan.n_chunks}", flush=True)
    g = api.enumerate_g(plan).cpu().numpy()
    assert int(g.sum(dtype=np.uint64)) == 1 << n
    np.testing.assert_array_equal(g.sum(axis=0).astype(object), closed_forms.binomial_marginal(n))
    np.testing.assert_array_equal(g, g[:, ::-1])
    np.testing.assert_array_equal(api.enumerate_symmetric(plan).cpu().numpy(), g)
    parts = torch.zeros((plan.n_e, plan.n_m), dtype=torch.uint64, device="cuda")
    cuts = sorted({0, plan.n_chunks, *[int(rng.next() % (plan.n_chunks + 1)) for _ in range(3)]})
    for a, b in zip(cuts[:-1], cuts[1:]):
        api.enumerate_range(plan, a, b - a, parts)
    np.testing.assert_array_equal(parts.cpu().numpy(), g)
