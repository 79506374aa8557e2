"""The autograd workload on its own inputs: log Z(T, h, J) of the 6x6 torus,
the J = 1 3x3x3 cube and the seeded +-J 3x3x3 cube, on the 64 x 64 grid
T = linspace(0.5, 5, 64), h = linspace(-1, 1, 64), through the autograd
Function, against the oracle:

  * log Z and the five (T, h) derivatives element by element (differentiating
    Eq. (2) with H = E - h M from Eq. (1));
  * the gradient of a seeded random loss sum G log Z in T, h and every
    coupling (per-bond d log Z/dJ_b = <s_i s_j>/T from the oracle's bond
    split: brute force for the cubes, the transfer-matrix split for the
    torus), and d log Z/dJ_b at single grid points;
  * central finite differences with step 1e-5 in T, h and J of the oracle's
    log Z, at sampled grid points and bonds;
  * the heat capacity and susceptibility of a double backward against the
    oracle's centred moments, at every grid point.

Tolerances are forward error bounds: 1e-12 times the magnitude of the terms
each quantity sums or subtracts (the largest |H| for <H>, Var(H)/T^2 plus
the 4|<H>|/T that cancels in the double backward's C = d(T^2 d_T)/dT, ...),
1e-13 times sum |W| g for the per-bond sums over all configurations, and
1e-7 for finite differences (rounding ~eps |log Z|/delta, truncation
~delta^2)."""
import numpy as np
import pytest
import torch

from conftest import moment_scales
from oracle import grad, native, thermo
from paper_1110_2561_amd import lattice as L

pytestmark = pytest.mark.gpu

TOL = 1e-12      # FP64 evaluations from g
TOL_SUM = 1e-13  # per-bond sums over 2^N configurations, relative to sum |W| g
TOL_FD = 1e-7    # central differences, step 1e-5
DELTA = 1e-5

W_ = L.workload("autograd")
NAMES = ["torus6x6", "cube3", "cube3_pm"]
LATS = dict(zip(NAMES, W_["lattices"]))
T_GRID, H_GRID = W_["T"], W_["h"]

_REF = {}


def _ref(name):
    """(g, {bond: gp_b}) from the oracle: the cubes' full brute-force bond
    split; for the torus its transfer-matrix table and the split of one
    horizontal and one vertical bond (every bond of the uniform, edge-
    transitive torus has the same split)."""
    if name not in _REF:
        lat = LATS[name]
        print(f"oracle tables of {name} (N={lat.n_spins})", flush=True)
        if lat.kind == "square_torus":
            Jh, Jv = L.torus_coupling_grids(lat)
            g = native.tm_torus(Jh, Jv)
            split = {}
            for b, (d, x, y) in ((0, (0, 0, 0)), (1, (1, 0, 0))):
                g2, gp = native.tm_torus_bond_split(Jh, Jv, d, x, y)
                assert np.array_equal(g2, g)
                split[b] = gp
        else:
            g, gp = native.bond_split(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
            split = {b: gp[b] for b in range(lat.n_bonds)}
        _REF[name] = (g, split)
    return _REF[name]


@pytest.fixture(scope="module")
def ag():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1110_2561_amd import autograd as M
    return M


@pytest.fixture(scope="module")
def api():
    from paper_1110_2561_amd import api as A
    return A


_F = {}


def _model(ag, name):
    if name not in _F:
        _F[name] = ag.IsingLogZ(LATS[name])
    return _F[name]


def _grid_tensors(requires_grad=True):
    T = torch.tensor(T_GRID, dtype=torch.float64, device="cuda", requires_grad=requires_grad)
    h = torch.tensor(H_GRID, dtype=torch.float64, device="cuda", requires_grad=requires_grad)
    return T, h


def _moment_scales(g, S, N):
    return moment_scales(g, S, N, T_GRID, H_GRID)


@pytest.mark.parametrize("name", NAMES)
def test_workload_logz_and_grid_derivatives(ag, api, name):
    lat = LATS[name]
    g, _ = _ref(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = _model(ag, name)
    assert torch.equal(f.g.cpu(), torch.from_numpy(g.view(np.int64)).view(torch.uint64))   # the model's own table
    T, h = _grid_tensors(requires_grad=False)
    lz = f(T, h).cpu().numpy()
    np.testing.assert_allclose(lz, thermo.log_z(g, -S, N, T_GRID, H_GRID), rtol=TOL, atol=0)
    # the (T, h) derivatives the backward and double backward use, every grid point
    d = {k: v.cpu().numpy() for k, v in api.logz_derivatives(f.g, -S, N, T, h).items()}
    ref = grad.log_z_derivatives(g, -S, N, T_GRID, H_GRID)
    sc = _moment_scales(g, S, N)
    for k, v in ref.items():
        err = np.abs(d[k] - v)
        assert (err <= TOL * sc[k]).all(), (k, float((err / sc[k]).max()))


@pytest.mark.parametrize("name", NAMES)
def test_workload_gradient_of_random_loss(ag, name):
    # L = sum G log Z over the 64 x 64 grid, G seeded; dL/dT, dL/dh, dL/dJ
    lat = LATS[name]
    g, split = _ref(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = _model(ag, name)
    T, h = _grid_tensors()
    J = f.couplings()
    G = np.random.default_rng(64).standard_normal((T_GRID.size, H_GRID.size))
    gT, gh, gJ = (x.cpu().numpy() for x in torch.autograd.grad((f(T, h, J) * torch.from_numpy(G).cuda()).sum(),
                                                                (T, h, J)))
    d = grad.log_z_derivatives(g, -S, N, T_GRID, H_GRID)
    sc = _moment_scales(g, S, N)
    assert (np.abs(gT - (G * d["d_T"]).sum(1)) <= TOL * (np.abs(G) * sc["d_T"]).sum(1)).all()
    assert (np.abs(gh - (G * d["d_h"]).sum(0)) <= TOL * (np.abs(G) * sc["d_h"]).sum(0)).all()
    # per bond: sum over configurations of W s_i s_j, W the oracle's bin weights of G
    Wref = grad.bin_weights(g, -S, N, T_GRID, H_GRID, G)
    bound = TOL_SUM * (np.abs(Wref) * g.astype(np.float64)).sum()
    bonds = sorted(split)
    refJ = grad.bond_grad_from_weights(g, np.stack([split[b] for b in bonds]), Wref)
    err = np.abs(gJ[bonds] - refJ)
    assert (err <= bound).all(), (float(err.max()), bound)
    if lat.kind == "square_torus":      # every bond of the uniform torus has the same sum
        assert (np.abs(gJ - refJ[0]) <= 2 * bound).all()


@pytest.mark.parametrize("name", NAMES)
def test_workload_bond_derivatives_at_single_points(ag, name):
    # d log Z(T_a, h_c)/dJ_b at single grid points (the loss selects one point),
    # against <s_i s_j>/T from the oracle's bond split
    lat = LATS[name]
    g, split = _ref(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = _model(ag, name)
    T, h = _grid_tensors(requires_grad=False)
    J = f.couplings()
    bonds = sorted(split)
    gp = np.stack([split[b] for b in bonds])
    for a, c in ((0, 0), (0, 40), (13, 31), (29, 32), (47, 5), (63, 63)):
        sel = torch.zeros((T_GRID.size, H_GRID.size), dtype=torch.float64, device="cuda")
        sel[a, c] = 1.0
        (gJ,) = torch.autograd.grad((f(T, h, J) * sel).sum(), J)
        ref = grad.bond_grad(g, gp, -S, N, [T_GRID[a]], [H_GRID[c]])[:, 0, 0]
        # the sum over configurations of p s_i s_j / T: sum |W| g = 1 / T
        bound = TOL_SUM / T_GRID[a]
        err = np.abs(gJ.cpu().numpy()[bonds] - ref)
        assert (err <= bound).all(), ((a, c), float(err.max()))


def _fd_points():
    return ((0, 0), (5, 20), (21, 43), (31, 31), (44, 2), (63, 60))


@pytest.mark.parametrize("name", NAMES)
def test_workload_central_finite_differences(ag, name):
    lat = LATS[name]
    g, split = _ref(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = _model(ag, name)
    bonds = sorted(split)
    if len(bonds) > 8:      # a sample of the cube's bonds, both signs of a +-J cube
        bonds = bonds[::10] + [b for b in bonds if lat.bond_J[b] < 0][:2]
    J = f.couplings()
    for a, c in _fd_points():
        t0, h0 = float(T_GRID[a]), float(H_GRID[c])
        T = torch.tensor([t0], dtype=torch.float64, device="cuda", requires_grad=True)
        h = torch.tensor([h0], dtype=torch.float64, device="cuda", requires_grad=True)
        gT, gh, gJ = (x.cpu().numpy() for x in torch.autograd.grad(f(T, h, J).sum(), (T, h, J)))

        def lz(t, hh):
            return float(thermo.log_z(g, -S, N, [t], [hh])[0, 0])

        fdT = (lz(t0 + DELTA, h0) - lz(t0 - DELTA, h0)) / (2 * DELTA)
        fdh = (lz(t0, h0 + DELTA) - lz(t0, h0 - DELTA)) / (2 * DELTA)
        assert gT[0] == pytest.approx(fdT, rel=TOL_FD), (a, c)
        assert gh[0] == pytest.approx(fdh, rel=TOL_FD, abs=TOL_FD * N / t0), (a, c)
        for b in bonds:      # J_b +- 1e-5 is not an integer: the oracle's bond split evaluates it
            fd = (grad.log_z_shifted(g, split[b], -S, N, t0, h0, DELTA)
                  - grad.log_z_shifted(g, split[b], -S, N, t0, h0, -DELTA)) / (2 * DELTA)
            assert gJ[b] == pytest.approx(fd, rel=TOL_FD, abs=TOL_FD / t0), (a, c, b)


@pytest.mark.parametrize("name", NAMES)
def test_workload_double_backward_heat_capacity_and_susceptibility(ag, name):
    # C = d<H>/dT with <H> = T^2 d log Z/dT, per h column; chi = d<M>/dh with
    # <M> = T d log Z/dh, per T row; every point of the 64 x 64 grid
    lat = LATS[name]
    g, _ = _ref(name)
    S, N = lat.abs_coupling_sum, lat.n_spins
    f = _model(ag, name)
    sc = _moment_scales(g, S, N)
    Tt = torch.tensor(T_GRID, dtype=torch.float64, device="cuda", requires_grad=True)
    C = np.empty((T_GRID.size, H_GRID.size))
    H = np.empty_like(C)
    for c, h0 in enumerate(H_GRID):
        hc = torch.tensor([h0], dtype=torch.float64, device="cuda")
        (dT,) = torch.autograd.grad(f(Tt, hc).sum(), Tt, create_graph=True)
        Hc = Tt * Tt * dT
        C[:, c] = torch.autograd.grad(Hc.sum(), Tt)[0].cpu().numpy()
        H[:, c] = Hc.detach().cpu().numpy()
    hmax = S + np.abs(H_GRID)[None, :] * N
    assert (np.abs(H - sc["mH"]) <= TOL * hmax).all()
    # the chain rule adds 2<H>/T and subtracts it again inside T^2 d_TT
    T = T_GRID[:, None]
    err = np.abs(C - sc["C"])
    assert (err <= TOL * (sc["C"] + 4 * hmax / T)).all(), float((err / (sc["C"] + 4 * hmax / T)).max())
    ht = torch.tensor(H_GRID, dtype=torch.float64, device="cuda", requires_grad=True)
    chi = np.empty_like(C)
    for a, t0 in enumerate(T_GRID):
        Ta = torch.tensor([t0], dtype=torch.float64, device="cuda")
        (dh,) = torch.autograd.grad(f(Ta, ht).sum(), ht, create_graph=True)
        chi[a] = torch.autograd.grad((t0 * dh).sum(), ht)[0].cpu().numpy()
    np.testing.assert_allclose(chi, sc["chi"], rtol=TOL, atol=0)
