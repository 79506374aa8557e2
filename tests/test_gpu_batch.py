"""Batched persistent enumeration, batched moments and graph replay, against
the oracle (bit-exact tables, FP64 log Z and moments within 1e-12).

Every member of the batch256 workload is compared with an oracle table: the
square tori with the transfer matrix, the triangular patches with the banded
count, the 3x3x3 cubes with the brute force's stored tables
(tests/golden/batch256_cubes.npz, written by an oracle-only script)."""
import numpy as np
import pytest
import torch

from conftest import load_cube_goldens
from oracle import closed_forms, native, thermo
from paper_1110_2561_amd import lattice as L

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1110_2561_amd import api as A
    return A


def _bf(lat):
    return native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)


def _tri(N, Lx, seed):
    base = L.triangular_free(N, Lx)
    return L.triangular_free(N, Lx, L.choice_couplings(base.n_bonds, seed))


def small_batch():
    return [
        L.square_torus(4, 5, L.choice_couplings(40, 1)),
        L.Lattice(1, [], [], []),
        L.ring(9, L.pm_couplings(9, 3)),
        _tri(17, 4, 5),
        L.cubic_torus(2, L.choice_couplings(24, 6)),
        L.random_bond_lattice(13, 40, 7),
        L.Lattice(6, [], [], []),
        L.square_torus(3, 6),
        L.random_bond_lattice(20, 35, 9, values=(-1, 1)),
        L.square_torus(4, 4),
        _tri(19, 5, 11),
        L.Lattice(3, [0, 1], [1, 2], [2, -2]),
    ]


@pytest.mark.parametrize("tune", [None, {"prefix_bits": 4}, {"prefix_bits": 12, "replicas": 4},
                                  {"max_blocks": 3, "waves_per_block": 4}, {"tile_bits": 2}],
                         ids=["default", "pb4", "pb12-r4", "3blocks", "tile2"])
@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
def test_small_batch_bit_exact(api, tune, symmetric):
    lats = small_batch()
    plan = api.BatchPlan(lats, api.Tune(**tune) if tune else None)
    stale = torch.full((int(plan.offsets[-1]),), 12345, dtype=torch.int64, device="cuda").view(torch.uint64)
    g = api.batch_enumerate(plan, out=stale, symmetric=symmetric)
    torch.cuda.synchronize()
    g_host = g.cpu()
    for i, lat in enumerate(lats):
        print(f"member {i}: {lat.kind} N={lat.n_spins}", flush=True)
        np.testing.assert_array_equal(plan.table(g_host, i).numpy(), _bf(lat))


@pytest.fixture(scope="module")
def b256():
    """The batch256 workload and the oracle's table of every member."""
    w = L.workload("batch256")
    cubes = load_cube_goldens()
    refs = []
    for i, lat in enumerate(w["lattices"]):
        if lat.kind == "square_torus":
            refs.append(native.tm_torus(*L.torus_coupling_grids(lat)))
        elif lat.kind == "triangular_free":           # bandwidth <= 7: the banded count
            refs.append(native.band_count(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J))
        else:                                         # 3x3x3 cube: stored brute-force table
            refs.append(cubes[i])
    return w, refs


def _check_moments(out, i, ref, lat, T, h, what):
    S, N = lat.abs_coupling_sum, lat.n_spins
    lz = thermo.log_z(ref, -S, N, T, h)
    mE, mM, C, chi = thermo.moments(ref, -S, N, T, h)
    msg = f"{what}: member {i} ({lat.kind}, N={N})"
    np.testing.assert_allclose(out["log_z"][i], lz, rtol=RTOL, atol=0, err_msg=msg)
    np.testing.assert_allclose(out["mean_E"][i], mE, rtol=RTOL, atol=RTOL * max(S, 1), err_msg=msg)
    np.testing.assert_allclose(out["mean_M"][i], mM, rtol=RTOL, atol=RTOL * N, err_msg=msg)
    np.testing.assert_allclose(out["heat_capacity"][i], C, rtol=RTOL, atol=1e-300, err_msg=msg)
    np.testing.assert_allclose(out["susceptibility"][i], chi, rtol=RTOL, atol=1e-300, err_msg=msg)


def test_batch256_parity(api, b256):
    w, refs = b256
    lats = w["lattices"]
    plan = api.BatchPlan(lats)
    g = api.batch_enumerate(plan)
    torch.cuda.synchronize()
    g_host = g.cpu()
    for i, lat in enumerate(lats):
        t = plan.table(g_host, i).numpy()
        N = lat.n_spins
        # properties that hold at any size
        assert int(t.sum()) == 1 << N, i
        np.testing.assert_array_equal(t.sum(axis=0).astype(object), closed_forms.binomial_marginal(N))
        np.testing.assert_array_equal(t, t[:, ::-1])
        # every member against the oracle, bit for bit
        np.testing.assert_array_equal(t, refs[i], err_msg=f"member {i} ({lat.kind}, N={N})")


def test_batch256_moments_match_oracle(api, b256):
    # the GPU's own batched tables and batched moments on the workload's
    # 64 x 3 grid, against the oracle's FP64 evaluation of the oracle tables
    w, refs = b256
    lats, T, h = w["lattices"], w["T"], w["h"]
    plan = api.BatchPlan(lats)
    g = api.batch_enumerate(plan)
    out = {k: v.cpu().numpy() for k, v in api.batch_moments(plan, g, T, h).items()}
    for i, lat in enumerate(lats):
        _check_moments(out, i, refs[i], lat, T, h, "batched moments")


def test_batch256_halved_equals_full(api):
    # every member with two or more chunks walks only its configurations with
    # the top spin up, then mirrors: the tables are identical to the full run
    lats = L.workload("batch256")["lattices"]
    plan = api.BatchPlan(lats)
    full = api.batch_enumerate(plan).cpu()
    half = api.batch_enumerate(plan, symmetric=True).cpu()
    assert torch.equal(full, half)


def test_batch_matches_single_lattice_path(api):
    # every member of batch256 equals its own single-lattice run
    lats = L.workload("batch256")["lattices"]
    plan = api.BatchPlan(lats)
    g = api.batch_enumerate(plan).cpu()
    for i, lat in enumerate(lats):
        p1 = api.Plan(lat)
        single = api.enumerate_g(p1).cpu()
        assert torch.equal(plan.table(g, i), single), i


def test_batch_moments_match_oracle(api):
    lats = small_batch()
    plan = api.BatchPlan(lats)
    T = np.linspace(0.5, 5.0, 16)
    h = np.array([-0.5, 0.0, 0.25])
    refs = [_bf(l) for l in lats]
    # evaluate on the oracle's tables so only the FP64 path differs
    flat = np.concatenate([r.reshape(-1) for r in refs])
    g = torch.from_numpy(flat.view(np.int64)).view(torch.uint64).cuda()
    out = api.batch_moments(plan, g, T, h)
    torch.cuda.synchronize()
    for i, lat in enumerate(lats):
        S, N = lat.abs_coupling_sum, lat.n_spins
        lz = thermo.log_z(refs[i], -S, N, T, h)
        mE, mM, C, chi = thermo.moments(refs[i], -S, N, T, h)
        np.testing.assert_allclose(out["log_z"][i].cpu().numpy(), lz, rtol=1e-12, atol=1e-13)
        np.testing.assert_allclose(out["mean_E"][i].cpu().numpy(), mE, rtol=1e-12, atol=1e-12 * max(S, 1))
        np.testing.assert_allclose(out["mean_M"][i].cpu().numpy(), mM, rtol=1e-12, atol=1e-12 * N)
        np.testing.assert_allclose(out["heat_capacity"][i].cpu().numpy(), C, rtol=RTOL, atol=1e-300)
        np.testing.assert_allclose(out["susceptibility"][i].cpu().numpy(), chi, rtol=RTOL, atol=1e-300)


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
def test_graph_replays_equal_eager(api, b256, symmetric):
    w, refs = b256
    lats, T, h = w["lattices"], w["T"], w["h"]
    plan = api.BatchPlan(lats)
    eager_g = api.batch_enumerate(plan)
    eager = api.batch_moments(plan, eager_g, T, h)
    torch.cuda.synchronize()
    graph = api.BatchGraph(plan, T, h, symmetric=symmetric)
    for rep in range(3):
        graph.g_all.fill_(7)                       # stale contents must be overwritten
        for v in graph.outs.values():
            v.fill_(float("nan"))
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(graph.g_all.cpu(), eager_g.cpu()), rep
        for k, v in eager.items():
            assert torch.equal(torch.nan_to_num(graph.outs[k], 1.5).cpu(), torch.nan_to_num(v, 1.5).cpu()), (rep, k)
        if rep == 0:      # the replay's results against the oracle
            g_host = graph.g_all.cpu()
            outs = {k: v.cpu().numpy() for k, v in graph.outs.items()}
            for i, lat in enumerate(lats):
                np.testing.assert_array_equal(plan.table(g_host, i).numpy(), refs[i], err_msg=f"member {i}")
                _check_moments(outs, i, refs[i], lat, T, h, "graph replay")
        # eager work between replays
        api.batch_enumerate(plan, out=eager_g)
        torch.cuda.synchronize()


def test_batch_errors(api):
    with pytest.raises(api.IsingError):
        api.BatchPlan([])
    with pytest.raises(api.IsingError, match="member 1"):
        api.BatchPlan([L.ring(5), L.Lattice(3, [0], [0], [1])])


def test_autotuner_picks_a_valid_tune_and_caches_it(api, tmp_path, monkeypatch):
    from paper_1110_2561_amd import autotune
    monkeypatch.setenv("ISING_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    lats = small_batch()
    cands = [api.Tune(), api.Tune(inner_bits=10), api.Tune(replicas=4)]
    tune, timings = autotune.autotune_batch(lats, candidates=cands, reps=1)
    assert tune in cands and len(timings) == 3 and all(t > 0 for t in timings.values())
    assert (tmp_path / "tune.json").exists()
    again, t2 = autotune.autotune_batch(lats, candidates=cands, reps=1)   # from the cache
    assert again == tune and t2 == timings
    g = api.batch_enumerate(api.BatchPlan(lats, tune)).cpu()              # the choice is exact too
    plan = api.BatchPlan(lats)
    for i, lat in enumerate(lats):
        np.testing.assert_array_equal(plan.table(g, i).numpy(), _bf(lat))
