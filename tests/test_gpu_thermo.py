"""Parity of the FP64 log Z / moments kernel with the oracle's evaluation.

Tolerance: 1e-12 relative (FP64 log-sum-exp over <= 10^4 bins; both sides
round differently only in summation order), absolute 1e-12 * N where the
exact value is 0 (<M> at h = 0).  C and chi are centred sums of non-negative
terms, so the same bound holds for them.
"""
import numpy as np
import pytest
import torch

from oracle import native, thermo
from paper_1110_2561_amd import lattice as L

pytestmark = pytest.mark.gpu

RTOL = 1e-12


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1110_2561_amd import api as A
    return A


def _ref_g(lat):
    if lat.kind == "square_torus" and lat.n_spins > 24:
        return native.tm_torus(*L.torus_coupling_grids(lat))
    return native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)


@pytest.mark.parametrize("name", ["torus4x4", "torus6x6", "torus8x5_pm"])
def test_logz_and_moments_match_oracle(api, name):
    w = L.workload(name)
    lat, T, h = w["lattice"], w["T"], w["h"]
    g_ref = _ref_g(lat)
    # evaluate both on the same (oracle) table, so only the FP64 path differs
    g = torch.from_numpy(g_ref.view(np.int64)).view(torch.uint64).cuda()
    S, N = lat.abs_coupling_sum, lat.n_spins
    out = api.moments(g, -S, N, T, h)
    lz = api.log_z(g, -S, N, T, h)
    torch.cuda.synchronize()
    ref_lz = thermo.log_z(g_ref, -S, N, T, h)
    mE, mM, C, chi = thermo.moments(g_ref, -S, N, T, h)
    np.testing.assert_allclose(lz.cpu().numpy(), ref_lz, rtol=RTOL, atol=0)
    np.testing.assert_allclose(out["log_z"].cpu().numpy(), ref_lz, rtol=RTOL, atol=0)
    np.testing.assert_allclose(out["mean_E"].cpu().numpy(), mE, rtol=RTOL, atol=RTOL * S)
    np.testing.assert_allclose(out["mean_M"].cpu().numpy(), mM, rtol=RTOL, atol=RTOL * N)
    np.testing.assert_allclose(out["heat_capacity"].cpu().numpy(), C, rtol=RTOL, atol=1e-300)
    np.testing.assert_allclose(out["susceptibility"].cpu().numpy(), chi, rtol=RTOL, atol=1e-300)


@pytest.mark.parametrize("nT,nh", [(1, 1), (7, 5), (3, 9), (13, 2)])
def test_ragged_grids(api, nT, nh):
    # grids whose temperature count is not a multiple of a block's waves and
    # whose field count is odd (a wave's second field slot unused), on the
    # +-J 8x5 table; the batched form on the same grid with two small members
    lat = L.workload("torus8x5_pm")["lattice"]
    g_ref = _ref_g(lat)
    g = torch.from_numpy(g_ref.view(np.int64)).view(torch.uint64).cuda()
    S, N = lat.abs_coupling_sum, lat.n_spins
    rng = np.random.default_rng(nT * 100 + nh)
    T = np.sort(rng.uniform(0.3, 6.0, nT))
    h = rng.uniform(-2.0, 2.0, nh)
    out = api.moments(g, -S, N, T, h)
    ref_lz = thermo.log_z(g_ref, -S, N, T, h)
    mE, mM, C, chi = thermo.moments(g_ref, -S, N, T, h)
    np.testing.assert_allclose(out["log_z"].cpu().numpy(), ref_lz, rtol=RTOL, atol=0)
    np.testing.assert_allclose(out["mean_E"].cpu().numpy(), mE, rtol=RTOL, atol=RTOL * S)
    np.testing.assert_allclose(out["mean_M"].cpu().numpy(), mM, rtol=RTOL, atol=RTOL * N)
    np.testing.assert_allclose(out["heat_capacity"].cpu().numpy(), C, rtol=RTOL, atol=1e-300)
    np.testing.assert_allclose(out["susceptibility"].cpu().numpy(), chi, rtol=RTOL, atol=1e-300)
    members = [L.square_torus(3, 4, L.pm_couplings(24, 5)), L.square_torus(4, 5, L.pm_couplings(40, 6))]
    batch = api.BatchPlan(members)
    tables = api.batch_enumerate(batch)
    bm = api.batch_moments(batch, tables, T, h)
    for k, lt in enumerate(members):
        gr = native.count_all(lt.n_spins, lt.bond_i, lt.bond_j, lt.bond_J)
        ref = thermo.log_z(gr, -lt.abs_coupling_sum, lt.n_spins, T, h)
        np.testing.assert_allclose(bm["log_z"][k].cpu().numpy(), ref, rtol=RTOL, atol=0)
        refC = thermo.moments(gr, -lt.abs_coupling_sum, lt.n_spins, T, h)[2]
        np.testing.assert_allclose(bm["heat_capacity"][k].cpu().numpy(), refC, rtol=RTOL, atol=1e-300)


def test_table_with_more_bins_than_the_lds_stage(api):
    # A 22-spin triangular patch with 8 widely spaced couplings has ~8300
    # nonzero bins, more than the 4096 the thermo kernels stage in LDS, so they
    # read the dense table in place.  Enumerated on the GPU (bit-exact against
    # the banded count), then log Z, moments and derivatives against the oracle.
    from conftest import moment_scales
    from oracle import grad
    base = L.triangular_free(22, 5)
    lat = L.triangular_free(22, 5, L.choice_couplings(base.n_bonds, 77, (-37, -11, 3, 23, -7, 13, 31, -19)))
    g_ref = native.band_count(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    assert np.count_nonzero(g_ref) > 4096
    plan = api.Plan(lat)
    g = api.enumerate_g(plan)
    np.testing.assert_array_equal(g.cpu().numpy(), g_ref)
    S, N = lat.abs_coupling_sum, lat.n_spins
    T = np.linspace(0.5, 5.0, 24)
    h = np.array([-1.0, 0.0, 0.3, 2.0, 5.0])
    out = {k: v.cpu().numpy() for k, v in api.moments(g, -S, N, T, h).items()}
    ref_lz = thermo.log_z(g_ref, -S, N, T, h)
    mE, mM, C, chi = thermo.moments(g_ref, -S, N, T, h)
    np.testing.assert_allclose(api.log_z(g, -S, N, T, h).cpu().numpy(), ref_lz, rtol=RTOL, atol=0)
    np.testing.assert_allclose(out["log_z"], ref_lz, rtol=RTOL, atol=0)
    np.testing.assert_allclose(out["mean_E"], mE, rtol=RTOL, atol=RTOL * S)
    np.testing.assert_allclose(out["mean_M"], mM, rtol=RTOL, atol=RTOL * N)
    np.testing.assert_allclose(out["heat_capacity"], C, rtol=RTOL, atol=1e-300)
    np.testing.assert_allclose(out["susceptibility"], chi, rtol=RTOL, atol=1e-300)
    d = {k: v.cpu().numpy() for k, v in api.logz_derivatives(g, -S, N, T, h).items()}
    sc = moment_scales(g_ref, S, N, T, h)
    for k, v in grad.log_z_derivatives(g_ref, -S, N, T, h).items():
        assert (np.abs(d[k] - v) <= RTOL * sc[k]).all(), k
    # the batched kernel reads it in place too
    bp = api.BatchPlan([lat, L.square_torus(4, 4)])
    gb = api.batch_enumerate(bp)
    ob = {k: v.cpu().numpy() for k, v in api.batch_moments(bp, gb, T, h).items()}
    np.testing.assert_array_equal(bp.table(gb.cpu(), 0).numpy(), g_ref)
    np.testing.assert_allclose(ob["log_z"][0], ref_lz, rtol=RTOL, atol=0)
    np.testing.assert_allclose(ob["heat_capacity"][0], C, rtol=RTOL, atol=1e-300)
    np.testing.assert_allclose(ob["susceptibility"][0], chi, rtol=RTOL, atol=1e-300)


def test_end_to_end_4x4_from_gpu_table(api):
    w = L.workload("torus4x4")
    lat = w["lattice"]
    plan = api.Plan(lat)
    g = api.enumerate_g(plan)
    lz = api.log_z(g, plan.e_min, lat.n_spins, w["T"], w["h"]).cpu().numpy()
    ref = thermo.log_z(native.count_all(16, lat.bond_i, lat.bond_j, lat.bond_J), -32, 16, w["T"], w["h"])
    np.testing.assert_allclose(lz, ref, rtol=RTOL, atol=0)


def test_bad_temperatures_and_empty_table(api):
    lat = L.square_torus(3, 3)
    plan = api.Plan(lat)
    g = api.enumerate_g(plan)
    out = api.moments(g, plan.e_min, 9, [0.0, -1.0, float("inf"), 1.0], [0.0])
    lz = out["log_z"].cpu().numpy()[:, 0]
    assert np.isnan(lz[:3]).all() and np.isfinite(lz[3])
    z = torch.zeros_like(g)
    out = api.moments(z, plan.e_min, 9, [1.0], [0.0, 0.5])
    assert np.isneginf(out["log_z"].cpu().numpy()).all()
    assert np.isnan(out["mean_E"].cpu().numpy()).all()


def test_thermo_argument_errors(api):
    g = torch.zeros((19, 10), dtype=torch.uint64, device="cuda")
    with pytest.raises(api.IsingError):
        api.log_z(g, -9, 8, [1.0], [0.0])        # n_m != N + 1
    empty = api.log_z(g, -9, 9, [], [0.0])
    assert empty.shape == (0, 1)


def test_command_line_table_and_thermo(api, tmp_path):
    """The command line (run in-process): the 4x4 table it writes is Table 1,
    its log Z matches the oracle, and the +-J 4x5 halved run writes the
    brute-force table."""
    import json

    from conftest import load_table1
    from paper_1110_2561_amd import __main__ as cli
    from paper_1110_2561_amd import table
    out, th = tmp_path / "g.txt", tmp_path / "th.json"
    assert cli.main(["torus:4x4", "--table", str(out), "--T", "0.5:5:4", "--h", "0,0.1", "--thermo", str(th)]) == 0
    assert {(e, m): c for c, m, e in table.read(str(out))} == load_table1()
    d = json.loads(th.read_text())
    lat = L.square_torus(4, 4)
    g = native.count_all(16, lat.bond_i, lat.bond_j, lat.bond_J)
    ref = thermo.log_z(g, -32, 16, np.array(d["T"]), np.array(d["h"]))
    np.testing.assert_allclose(np.array(d["log_z"]), ref, rtol=1e-12)
    assert cli.main(["torus:4x5", "--pm", "5", "--symmetric", "--table", str(out)]) == 0
    lat = L.square_torus(4, 5, L.pm_couplings(40, 5))
    g = native.count_all(20, lat.bond_i, lat.bond_j, lat.bond_J)
    assert table.read(str(out)) == table.rows(g, -40, 20)
