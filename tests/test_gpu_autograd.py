"""Derivatives of log Z on the GPU against the oracle: the (T, h) derivative
kernel, the per-bin weights, the per-bond backward (recomputed enumeration),
the autograd Function (first derivatives, finite differences, double
backward for C and chi), and the 6x6 torus against Kaufman's closed form."""
import zlib

import mpmath as mp
import numpy as np
import pytest
import torch

from conftest import moment_scales
from oracle import closed_forms, grad, native, thermo
from paper_1110_2561_amd import lattice as L

pytestmark = pytest.mark.gpu

# Forward error bounds: FP64 evaluations from g within 1e-12 of the magnitude
# of the terms each formula combines (moment_scales); sums over all 2^N
# configurations within 1e-13 of sum |W| g.
TOL = 1e-12
TOL_SUM = 1e-13


@pytest.fixture(scope="module")
def api():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1110_2561_amd import api as A
    return A


@pytest.fixture(scope="module")
def ag():
    from paper_1110_2561_amd import autograd as M
    return M


def _tri(N, Lx, seed):
    base = L.triangular_free(N, Lx)
    return L.triangular_free(N, Lx, L.choice_couplings(base.n_bonds, seed))


LATS = {
    "torus4x4": L.square_torus(4, 4),
    "cubic3_pm": L.cubic_torus(3, L.choice_couplings(81, 6)),
    "tri19": _tri(19, 5, 11),
    "random14_4cls": L.random_bond_lattice(14, 40, 7, values=(-2, -1, 1, 2)),
    "ring9": L.ring(9, L.pm_couplings(9, 3)),
    "repeated": L.Lattice(6, [0, 1, 1, 2, 4, 0, 5], [1, 2, 2, 3, 5, 5, 3], [1, -2, 3, 1, -1, 2, 2]),
    "tiny3": L.Lattice(3, [0, 1], [1, 2], [2, -1]),
    "torus4x5_pm": L.square_torus(4, 5, L.pm_couplings(40, 5)),
}

_SPLIT = {}


def _split(name):
    if name not in _SPLIT:
        lat = LATS[name]
        print(f"oracle bond split {name} N={lat.n_spins}", flush=True)
        _SPLIT[name] = native.bond_split(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    return _SPLIT[name]


def _dev_table(g):
    return torch.from_numpy(np.ascontiguousarray(g).view(np.int64)).view(torch.uint64).cuda()


T_GRID = np.array([0.6, 1.1, 2.269, 3.7])
H_GRID = np.array([-0.7, 0.0, 0.35])


@pytest.mark.parametrize("name", ["torus4x4", "random14_4cls", "ring9"])
def test_logz_derivatives_match_oracle(api, name):
    lat = LATS[name]
    g, _ = _split(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    out = api.logz_derivatives(_dev_table(g), -S, N, T_GRID, H_GRID)
    ref = grad.log_z_derivatives(g, -S, N, T_GRID, H_GRID)
    np.testing.assert_allclose(out["log_z"].cpu().numpy(), thermo.log_z(g, -S, N, T_GRID, H_GRID), rtol=1e-13)
    sc = moment_scales(g, S, N, T_GRID, H_GRID)
    for k, v in ref.items():
        err = np.abs(out[k].cpu().numpy() - v)
        assert (err <= TOL * sc[k]).all(), (k, float((err / sc[k]).max()))


@pytest.mark.parametrize("name", ["torus4x4", "cubic3_pm", "ring9"])
def test_bin_weights_match_oracle(api, name):
    lat = LATS[name]
    g, _ = _split(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    G = np.random.default_rng(1).standard_normal((T_GRID.size, H_GRID.size))
    lz = api.log_z(_dev_table(g), -S, N, T_GRID, H_GRID)
    W = api.bin_weights(_dev_table(g), -S, N, T_GRID, H_GRID, lz, torch.from_numpy(G).cuda()).cpu().numpy()
    ref = grad.bin_weights(g, -S, N, T_GRID, H_GRID, G)
    np.testing.assert_allclose(W, ref, rtol=1e-12, atol=1e-15 * np.abs(ref).max())


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
@pytest.mark.parametrize("name", list(LATS))
def test_bond_backward_matches_oracle(api, name, symmetric):
    lat = LATS[name]
    g, gp = _split(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    # a weight table with structure on every realised bin (and junk on empty ones,
    # which no configuration reads)
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    W = rng.standard_normal(g.shape) * np.exp(-rng.uniform(0, 3, g.shape))
    plan = api.Plan(lat)
    print(f"{name}: N={N} tile={plan.tile_bits} bonds={lat.n_bonds}", flush=True)
    dJ = api.bond_backward(plan, torch.from_numpy(W).cuda(), symmetric=symmetric).cpu().numpy()
    ref = grad.bond_grad_from_weights(g, gp, np.where(g > 0, W, 0.0))
    scale = (np.abs(W) * g.astype(np.float64)).sum()
    np.testing.assert_allclose(dJ, ref, rtol=0, atol=1e-13 * scale)


def _bond_kinds(plan, lat):
    """Where each bond's two spins sit in the backward walk: inner (tile and up
    to 2 middle bits), offset (the next 10 bits, fixed per thread), block (up
    to 8 bits, fixed per block) or hi (the rest, walked in Gray order)."""
    N, TJ = lat.n_spins, plan.tile_bits
    above = max(0, N - TJ - 10)
    s = min(8, above)
    kb = TJ + min(2, above - s)

    def kind(bit):
        if bit < kb:
            return "inner"
        if bit < kb + 10:
            return "offset"
        return "block" if bit < kb + 10 + s else "hi"

    out = {}
    for b, (i, j) in enumerate(zip(lat.bond_i, lat.bond_j)):
        a, c = sorted((int(plan.bit_of_site[i]), int(plan.bit_of_site[j])))
        out.setdefault(kind(a) + "-" + kind(c), []).append(b)
    return out


def _torus_bond(lat, b):
    Lx = lat.dims[0]
    u, d = divmod(b, 2)
    return d, u % Lx, u // Lx


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
def test_torus8x5_pm_backward_sampled_bonds_match_transfer_matrix(api, symmetric):
    # The full 2^40 backward on the +-J 8x5 torus (12 hi bits: 4096 chunks per
    # thread), with a random weight table; two bonds of every kind of bit pair,
    # each against the oracle's transfer-matrix split of that bond.
    lat = L.workload("torus8x5_pm")["lattice"]
    Jh, Jv = L.torus_coupling_grids(lat)
    g = native.tm_torus(Jh, Jv)
    rng = np.random.default_rng(8_5)
    W = np.where(g > 0, rng.standard_normal(g.shape) * np.exp(-rng.uniform(0, 3, g.shape)), 0.0)
    plan = api.Plan(lat)
    kinds = _bond_kinds(plan, lat)
    print("8x5 bond kinds:", {k: len(v) for k, v in sorted(kinds.items())}, flush=True)
    assert {"inner-inner", "inner-offset", "inner-block", "inner-hi", "offset-offset", "offset-block",
            "offset-hi", "block-block", "block-hi", "hi-hi"} <= set(kinds)
    dJ = api.bond_backward(plan, torch.from_numpy(W).cuda(), symmetric=symmetric).cpu().numpy()
    scale = (np.abs(W) * g.astype(np.float64)).sum()
    for k in sorted(kinds):
        for b in kinds[k][:2]:
            g2, gp = native.tm_torus_bond_split(Jh, Jv, *_torus_bond(lat, b))
            assert np.array_equal(g2, g)
            ref = grad.bond_grad_from_weights(g, gp[None], W)[0]
            assert abs(dJ[b] - ref) <= 1e-13 * scale, (k, b, dJ[b], ref, scale)


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
@pytest.mark.parametrize("dims,seed,every", [((4, 8), 41, 1), ((8, 4), 42, 1), ((5, 6), 43, 7)])
def test_four_valued_tori_with_hi_bits_match_transfer_matrix(api, dims, seed, every, symmetric):
    # Tori of 30-32 spins with couplings in {-2, -1, 1, 2} (four coupling
    # classes): beyond 28 spins the walk has hi bits, so pairs with hi bits
    # take the summation by parts; every bond (every 7th on 5x6) against the
    # oracle's transfer-matrix split.
    lx, ly = dims
    lat = L.square_torus(lx, ly, L.choice_couplings(2 * lx * ly, seed, (-2, -1, 1, 2)))
    Jh, Jv = L.torus_coupling_grids(lat)
    g = native.tm_torus(Jh, Jv)
    rng = np.random.default_rng(seed)
    W = np.where(g > 0, rng.standard_normal(g.shape) * np.exp(-rng.uniform(0, 3, g.shape)), 0.0)
    plan = api.Plan(lat)
    kinds = _bond_kinds(plan, lat)
    print(f"{lx}x{ly}: N={lat.n_spins} bond kinds", {k: len(v) for k, v in sorted(kinds.items())}, flush=True)
    assert any(k.endswith("-hi") for k in kinds)
    dJ = api.bond_backward(plan, torch.from_numpy(W).cuda(), symmetric=symmetric).cpu().numpy()
    scale = (np.abs(W) * g.astype(np.float64)).sum()
    for b in range(0, lat.n_bonds, every):
        key = (dims, seed, b)
        if key not in _TM_SPLITS:
            g2, gp = native.tm_torus_bond_split(Jh, Jv, *_torus_bond(lat, b))
            assert np.array_equal(g2, g)
            _TM_SPLITS[key] = gp
        ref = grad.bond_grad_from_weights(g, _TM_SPLITS[key][None], W)[0]
        assert abs(dJ[b] - ref) <= 1e-13 * scale, (b, dJ[b], ref, scale)


_TM_SPLITS = {}   # transfer-matrix bond splits, shared by the full and halved cases


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
def test_torus6x6_backward_random_weights_equal_on_every_bond(api, symmetric):
    # On the edge-transitive 6x6 torus at uniform J every bond has the same
    # split table, so for any W(E, M) all 72 bond sums agree; one horizontal and
    # one vertical bond are checked against the transfer-matrix split.
    lat = L.square_torus(6, 6)
    Jh, Jv = L.torus_coupling_grids(lat)
    g = native.tm_torus(Jh, Jv)
    rng = np.random.default_rng(36)
    W = np.where(g > 0, rng.uniform(-1, 1, g.shape), 0.0)
    plan = api.Plan(lat)
    dJ = api.bond_backward(plan, torch.from_numpy(W).cuda(), symmetric=symmetric).cpu().numpy()
    scale = (np.abs(W) * g.astype(np.float64)).sum()
    np.testing.assert_allclose(dJ, dJ.mean(), rtol=0, atol=1e-13 * scale)
    for b in (0, 1):
        _, gp = native.tm_torus_bond_split(Jh, Jv, *_torus_bond(lat, b))
        ref = grad.bond_grad_from_weights(g, gp[None], W)[0]
        assert abs(dJ[b] - ref) <= 1e-13 * scale, (b, dJ[b], ref, scale)


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
@pytest.mark.parametrize("n,mid", [(22, 1), (23, 2), (26, 2), (19, 0), (12, 0)])
def test_bond_backward_middle_widths(api, n, mid, symmetric):
    # With a 3-bit tile the backward takes s = min(8, n - 13) block bits and
    # mid = min(2, n - 13 - s) middle bits (fewer on small lattices, to keep
    # 256 blocks); 26 spins leave 3 hi bits.  These sizes cover every middle
    # width, and with it every split of the spins between middle, offset,
    # block and hi bits.
    lat = L.random_bond_lattice(n, 3 * n, 100 + n, values=(-1, 1))
    assert mid == max(0, min(2, n - 13 - min(8, max(0, n - 13))))
    g, gp = native.bond_split(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    rng = np.random.default_rng(n)
    W = np.where(g > 0, rng.standard_normal(g.shape), 0.0)
    plan = api.Plan(lat, api.Tune(tile_bits=3))
    assert plan.tile_bits == 3
    dJ = api.bond_backward(plan, torch.from_numpy(W).cuda(), symmetric=symmetric).cpu().numpy()
    ref = grad.bond_grad_from_weights(g, gp, W)
    scale = (np.abs(W) * g.astype(np.float64)).sum()
    np.testing.assert_allclose(dJ, ref, rtol=0, atol=1e-13 * scale)


def test_bond_backward_is_reproducible_and_matches_small_tune(api):
    lat = LATS["cubic3_pm"]
    g, gp = _split("cubic3_pm")
    W = np.random.default_rng(5).uniform(-1, 1, g.shape)
    Wd = torch.from_numpy(W).cuda()
    a = api.bond_backward(api.Plan(lat), Wd)
    b = api.bond_backward(api.Plan(lat), Wd)
    assert torch.equal(a, b)                                   # fixed summation order
    c = api.bond_backward(api.Plan(lat, api.Tune(tile_bits=3)), Wd)   # another tile and walk
    np.testing.assert_allclose(c.cpu().numpy(), a.cpu().numpy(), rtol=1e-12, atol=1e-12 * np.abs(W).max() * 2 ** 27)


def test_bond_backward_edge_cases(api):
    # no bonds: nothing to do
    p0 = api.Plan(L.Lattice(5, [], [], []))
    assert api.bond_backward(p0, torch.zeros((1, 6), dtype=torch.float64, device="cuda")).numel() == 0
    # couplings of one pair that cancel: its spin product still has an average
    lat = L.Lattice(4, [0, 0, 1, 2], [1, 1, 2, 3], [1, -1, 2, -1])
    g, gp = native.bond_split(4, lat.bond_i, lat.bond_j, lat.bond_J)
    W = np.random.default_rng(8).uniform(0.5, 1.5, g.shape)
    dJ = api.bond_backward(api.Plan(lat), torch.from_numpy(W).cuda()).cpu().numpy()
    np.testing.assert_allclose(dJ, grad.bond_grad_from_weights(g, gp, np.where(g > 0, W, 0.0)), rtol=1e-14)
    assert dJ[0] == dJ[1] and dJ[0] != 0.0
    # N = 1 with no bonds, N = 2 with one bond
    lat = L.Lattice(2, [0], [1], [3])
    g, gp = native.bond_split(2, lat.bond_i, lat.bond_j, lat.bond_J)
    W = np.arange(g.size, dtype=np.float64).reshape(g.shape)
    dJ = api.bond_backward(api.Plan(lat), torch.from_numpy(W).cuda()).cpu().numpy()
    np.testing.assert_allclose(dJ, grad.bond_grad_from_weights(g, gp, np.where(g > 0, W, 0.0)), rtol=1e-15)
    # outputs of the wrong size, type or layout are refused before any launch
    plan = api.Plan(L.square_torus(4, 4))
    Wd = torch.zeros((plan.n_e, plan.n_m), dtype=torch.float64, device="cuda")
    for bad in (torch.zeros(31, dtype=torch.float64, device="cuda"),
                torch.zeros(32, dtype=torch.float32, device="cuda"),
                torch.zeros(64, dtype=torch.float64, device="cuda")[::2]):
        with pytest.raises(ValueError):
            api.bond_backward(plan, Wd, out=bad)
    gt = api.enumerate_g(plan)
    lz = api.log_z(gt, plan.e_min, 16, [1.0, 2.0], [0.0])
    G = torch.ones_like(lz)
    with pytest.raises(ValueError):
        api.bin_weights(gt, plan.e_min, 16, [1.0, 2.0], [0.0], lz, G,
                        out=torch.zeros((plan.n_e, plan.n_m - 1), dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        api.log_z(gt.t(), plan.e_min, 16, [1.0], [0.0])        # not contiguous


# --------------------------------------------------------------------------
# autograd
# --------------------------------------------------------------------------

def test_autograd_first_derivatives_match_oracle(ag):
    name = "cubic3_pm"
    lat = LATS[name]
    g, gp = _split(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = ag.IsingLogZ(lat)
    T = torch.tensor(T_GRID, device="cuda", requires_grad=True)
    h = torch.tensor(H_GRID, device="cuda", requires_grad=True)
    J = f.couplings()
    lz = f(T, h, J)
    np.testing.assert_allclose(lz.detach().cpu().numpy(), thermo.log_z(g, -S, N, T_GRID, H_GRID), rtol=1e-13)
    G = np.random.default_rng(3).standard_normal(lz.shape)
    gT, gh, gJ = torch.autograd.grad((lz * torch.from_numpy(G).cuda()).sum(), (T, h, J))
    d = grad.log_z_derivatives(g, -S, N, T_GRID, H_GRID)
    sc = moment_scales(g, S, N, T_GRID, H_GRID)
    assert (np.abs(gT.cpu().numpy() - (G * d["d_T"]).sum(1)) <= TOL * (np.abs(G) * sc["d_T"]).sum(1)).all()
    assert (np.abs(gh.cpu().numpy() - (G * d["d_h"]).sum(0)) <= TOL * (np.abs(G) * sc["d_h"]).sum(0)).all()
    refJ = (G[None] * grad.bond_grad(g, gp, -S, N, T_GRID, H_GRID)).sum(axis=(1, 2))
    Wref = grad.bin_weights(g, -S, N, T_GRID, H_GRID, G)
    bound = TOL_SUM * (np.abs(Wref) * g.astype(np.float64)).sum()
    assert (np.abs(gJ.cpu().numpy() - refJ) <= bound).all()


def test_autograd_matches_central_finite_differences(ag):
    name = "tri19"
    lat = LATS[name]
    g, gp = _split(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = ag.IsingLogZ(lat)
    T0, h0, d = 1.7, 0.3, 1e-5
    T = torch.tensor([T0], device="cuda", dtype=torch.float64, requires_grad=True)
    h = torch.tensor([h0], device="cuda", dtype=torch.float64, requires_grad=True)
    J = f.couplings()
    gT, gh, gJ = torch.autograd.grad(f(T, h, J).sum(), (T, h, J))
    lz = lambda t, hh: float(f(torch.tensor([t], device="cuda", dtype=torch.float64),   # noqa: E731
                               torch.tensor([hh], device="cuda", dtype=torch.float64))[0, 0])
    assert gT.item() == pytest.approx((lz(T0 + d, h0) - lz(T0 - d, h0)) / (2 * d), rel=1e-7)
    assert gh.item() == pytest.approx((lz(T0, h0 + d) - lz(T0, h0 - d)) / (2 * d), rel=1e-7)
    # couplings: J_b +- 1e-5 is not an integer, so the oracle's bond split evaluates it
    for b in range(0, lat.n_bonds, 7):
        fd = (grad.log_z_shifted(g, gp[b], -S, N, T0, h0, d) - grad.log_z_shifted(g, gp[b], -S, N, T0, h0, -d)) / (2 * d)
        assert gJ[b].item() == pytest.approx(fd, rel=1e-6, abs=1e-9), b


def test_double_backward_gives_heat_capacity_and_susceptibility(api, ag):
    name = "random14_4cls"
    lat = LATS[name]
    g, _ = _split(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = ag.IsingLogZ(lat)
    for h0 in (0.0, 0.45):
        T = torch.tensor(T_GRID, device="cuda", requires_grad=True)
        h = torch.tensor([h0], device="cuda", dtype=torch.float64, requires_grad=True)
        lz = f(T, h)
        dT, dh = torch.autograd.grad(lz.sum(), (T, h), create_graph=True)
        H = T * T * dT                         # <E - hM> per temperature
        C = torch.autograd.grad(H.sum(), T, retain_graph=True)[0]
        sc = moment_scales(g, S, N, T_GRID, [h0])
        Cref, chiref, hmax = sc["C"], sc["chi"], sc["hmax"][:, 0]
        assert (np.abs(H.detach().cpu().numpy() - sc["mH"][:, 0]) <= TOL * hmax).all()
        # C = 2T d_T + T^2 d_TT: the chain rule adds 2<H>/T and subtracts it inside T^2 d_TT
        cbound = TOL * (Cref[:, 0] + 4 * hmax / T_GRID)
        assert (np.abs(C.cpu().numpy() - Cref[:, 0]) <= cbound).all()
        # chi at each T separately (h has one point): <M> = T d log Z/dh
        for a, t in enumerate(T_GRID):
            Ta = torch.tensor([t], device="cuda", dtype=torch.float64)
            ha = torch.tensor([h0], device="cuda", dtype=torch.float64, requires_grad=True)
            (dha,) = torch.autograd.grad(f(Ta, ha).sum(), ha, create_graph=True)
            chi = torch.autograd.grad((t * dha).sum(), ha)[0]
            assert chi.item() == pytest.approx(chiref[a, 0], rel=TOL)
        mom = api.moments(_dev_table(g), -S, N, T_GRID, [h0])
        assert (np.abs(C.cpu().numpy() - mom["heat_capacity"][:, 0].cpu().numpy()) <= cbound).all()


def test_second_derivative_in_couplings_raises(ag):
    f = ag.IsingLogZ(LATS["torus4x4"])
    J = f.couplings()
    T = torch.tensor([2.0], device="cuda", dtype=torch.float64)
    (gJ,) = torch.autograd.grad(f(T, torch.tensor([0.0], device="cuda", dtype=torch.float64), J).sum(), J,
                                create_graph=True)
    with pytest.raises(RuntimeError, match="not implemented"):
        torch.autograd.grad(gJ.sum(), J)


def test_couplings_must_match_lattice(ag):
    f = ag.IsingLogZ(LATS["torus4x4"])
    J = f.couplings().detach().clone()
    J[0] = 0.5
    with pytest.raises(ValueError, match="integer couplings"):
        f(torch.tensor([1.0], device="cuda", dtype=torch.float64), torch.tensor([0.0], device="cuda",
                                                                                dtype=torch.float64), J)


# --------------------------------------------------------------------------
# 6x6 torus (2^36 configurations): per-bond gradients against Kaufman
# --------------------------------------------------------------------------

def test_torus6x6_bond_gradients_match_kaufman_and_sum_rule(api, ag):
    lat = L.square_torus(6, 6)
    f = ag.IsingLogZ(lat)
    T_list = np.array([1.5, 2.269, 3.0])
    h_list = np.array([0.0, 0.2])
    T = torch.tensor(T_list, device="cuda")
    h = torch.tensor(h_list, device="cuda")
    J = f.couplings()
    gref = native.tm_torus(*L.torus_coupling_grids(lat))
    for a, t in enumerate(T_list):
        for c, hh in enumerate(h_list):
            sel = torch.zeros((T_list.size, h_list.size), dtype=torch.float64, device="cuda")
            sel[a, c] = 1.0
            (gJ,) = torch.autograd.grad((f(T, h, J) * sel).sum(), J)
            gJ = gJ.cpu().numpy()
            # each bond's sum over configurations of p s_i s_j / T: sum |W| g = 1/T
            bound = TOL_SUM / t
            # edge-transitive torus at uniform J: every bond has the same gradient
            assert (np.abs(gJ - gJ.mean()) <= 2 * bound).all()
            # sum rule: sum_b J_b d log Z/dJ_b = -<E>/T, with <E> from the oracle's exact table
            mE, _, _, _ = thermo.moments(gref, -72, 36, [t], [hh])
            assert abs(float((lat.bond_J * gJ).sum()) + mE[0, 0] / t) <= 72 * bound + TOL * 72 / t
            if hh == 0.0:
                with mp.workdps(40):
                    dK = float(mp.diff(lambda Jv: closed_forms.kaufman_logz(6, 6, t / Jv), 1))
                assert (np.abs(gJ - dK / lat.n_bonds) <= bound).all()


def test_symmetric_backward_option_matches_full(ag):
    # IsingLogZ(symmetric_backward=True) gives the same per-bond gradient as the
    # full recomputation (+-J cube, random loss weights over a 5 x 3 grid).
    lat = LATS["cubic3_pm"]
    T = torch.tensor([0.8, 1.3, 2.0, 3.1, 4.5], dtype=torch.float64, device="cuda")
    h = torch.tensor([-0.4, 0.0, 0.9], dtype=torch.float64, device="cuda")
    G = torch.from_numpy(np.random.default_rng(3).standard_normal((5, 3))).cuda()
    out = []
    for sym in (False, True):
        f = ag.IsingLogZ(lat, symmetric_backward=sym)
        J = f.couplings()
        (gJ,) = torch.autograd.grad((f(T, h, J) * G).sum(), J)
        out.append(gJ.cpu().numpy())
    np.testing.assert_allclose(out[1], out[0], rtol=1e-12, atol=1e-13 * np.abs(out[0]).max())


@pytest.mark.parametrize("symmetric", [False, True], ids=["full", "halved"])
@pytest.mark.parametrize("grid", ["moderate", "strong_fields", "cold"])
def test_logz_backward_one_call_matches_separate_kernels(api, symmetric, grid):
    # ising_logz_backward issues the derivative, weight and per-bond kernels in
    # one call: its grad_J equals bin_weights + bond_backward, and grad_T,
    # grad_h are the derivative kernel's d_T, d_h contracted with G
    lat = L.square_torus(4, 6, L.pm_couplings(48, 9))
    plan = api.Plan(lat)
    g = api.enumerate_g(plan)
    # strong fields and low temperatures take the direct sum for some or all
    # (bin, T) terms of the factorised weights
    Tv, hv = {"moderate": ([0.7, 1.3, 2.2, 4.0], [-0.5, 0.0, 0.3]),
              "strong_fields": ([0.3, 0.5, 1.0, 3.0], [-40.0, 0.0, 25.0]),
              "cold": ([0.08, 0.1, 0.15, 0.2], [-0.5, 0.0, 0.3])}[grid]
    T = torch.tensor(Tv, dtype=torch.float64, device="cuda")
    h = torch.tensor(hv, dtype=torch.float64, device="cuda")
    lz = api.log_z(g, plan.e_min, lat.n_spins, T, h)
    G = torch.from_numpy(np.random.default_rng(11).standard_normal((4, 3))).cuda()
    gT, gh, gJ = api.logz_backward(plan, g, T, h, lz, G, symmetric=symmetric)
    W = api.bin_weights(g, plan.e_min, lat.n_spins, T, h, lz, G)
    # the one-call path forms the same weights by a factorised sum: equal up
    # to rounding of each term, so the bond sums agree within the backward's
    # bound relative to sum |W| g
    ref = api.bond_backward(plan, W, symmetric=symmetric).cpu().numpy()
    scale = (np.abs(W.cpu().numpy()) * g.cpu().numpy().astype(np.float64)).sum()
    assert (np.abs(gJ.cpu().numpy() - ref) <= 1e-13 * scale).all()
    d = api.logz_derivatives(g, plan.e_min, lat.n_spins, T, h)
    Gn, dT, dh = G.cpu().numpy(), d["d_T"].cpu().numpy(), d["d_h"].cpu().numpy()
    # the one-call path normalises by the forward's log Z in one pass, the
    # derivative kernel by the largest term in two: equal up to rounding of
    # the terms, |H| <= S + |h| N and |M| <= N
    Tn, hn, S, N = T.cpu().numpy()[:, None], h.cpu().numpy()[None, :], lat.abs_coupling_sum, lat.n_spins
    scT, sch = (S + np.abs(hn) * N) / Tn ** 2, N / Tn + 0 * hn
    assert (np.abs(gT.cpu().numpy() - (Gn * dT).sum(1)) <= 1e-13 * (np.abs(Gn) * scT).sum(1)).all()
    assert (np.abs(gh.cpu().numpy() - (Gn * dh).sum(0)) <= 1e-13 * (np.abs(Gn) * sch).sum(0)).all()
    if grid != "moderate":
        return
    # parts may be skipped; an empty grid gives zero gradients
    a, b, c = api.logz_backward(plan, g, T, h, lz, G, want=(False, True, False))
    assert a is None and c is None and torch.equal(b, gh)
    e0 = torch.empty((0, 3), dtype=torch.float64, device="cuda")
    zT, zh, zJ = api.logz_backward(plan, g, T[:0], h, e0, e0)
    assert zT.numel() == 0 and torch.equal(zh, torch.zeros_like(zh)) and torch.equal(zJ, torch.zeros_like(zJ))
    with pytest.raises(ValueError):
        api.logz_backward(plan, g, T, h, lz[:, :2], G)
