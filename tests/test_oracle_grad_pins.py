"""Pins of the oracle's derivative statistics (no GPU).

The bond-resolved counts and the derivative formulas are checked against
facts they do not compute themselves: exact integer identities, symmetry,
independent numpy enumeration (also with non-integer couplings), and
derivatives of the 1D ring and Kaufman torus closed forms taken by mpmath.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import closed_forms, grad, native, thermo
from paper_1110_2561_amd import lattice as L


def _split(lat):
    return native.bond_split(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)


def _numpy_configs(n):
    c = np.arange(1 << n)
    return ((c[:, None] >> np.arange(n)) & 1) * 2 - 1          # s[c][u]


LATS = [
    L.square_torus(4, 4),
    L.random_bond_lattice(10, 24, 3, values=(-2, -1, 1, 2)),
    L.Lattice(6, [0, 1, 1, 2, 4, 0, 5], [1, 2, 2, 3, 5, 5, 3], [1, -2, 3, 1, -1, 2, 2]),   # repeated pair (1, 2)
    L.ring(7, L.pm_couplings(7, 11)),
]


@pytest.mark.parametrize("lat", LATS, ids=lambda l: f"{l.kind}{l.n_spins}")
def test_split_counts_invariants(lat):
    g, gp = _split(lat)
    N = lat.n_spins
    np.testing.assert_array_equal(g, native.count_all(N, lat.bond_i, lat.bond_j, lat.bond_J))
    for b in range(lat.n_bonds):
        assert int(gp[b].sum()) == 1 << (N - 1)              # half the configurations agree
        np.testing.assert_array_equal(gp[b], gp[b][:, ::-1])  # global flip keeps s_i s_j
        assert (gp[b] <= g).all()


@pytest.mark.parametrize("lat", LATS, ids=lambda l: f"{l.kind}{l.n_spins}")
def test_split_counts_energy_identity(lat):
    # per bin: sum_b J_b * (sum of s_i s_j) = -E * g, in exact integers
    g, gp = _split(lat)
    S = lat.abs_coupling_sum
    sig = 2 * gp.astype(object) - g.astype(object)[None]
    lhs = sum(int(J) * sig[b] for b, J in enumerate(lat.bond_J))
    E = np.arange(-S, S + 1, dtype=object)[:, None]
    np.testing.assert_array_equal(lhs, -E * g.astype(object))


def test_split_counts_match_numpy_enumeration():
    lat = L.random_bond_lattice(9, 20, 5, values=(-1, 1, 2, 3))
    g, gp = _split(lat)
    s = _numpy_configs(9)
    sigma = s[:, lat.bond_i] * s[:, lat.bond_j]
    E = -(sigma * lat.bond_J).sum(axis=1)
    nup = (s > 0).sum(axis=1)
    S = lat.abs_coupling_sum
    for b in range(lat.n_bonds):
        ref = np.zeros_like(gp[b])
        np.add.at(ref, (E[sigma[:, b] > 0] + S, nup[sigma[:, b] > 0]), 1)
        np.testing.assert_array_equal(gp[b], ref)


# --------------------------------------------------------------------------
# bond correlations against closed forms
# --------------------------------------------------------------------------

@pytest.mark.parametrize("T,h", [(0.7, 0.0), (1.5, 0.0), (2.0, 0.3), (4.0, -0.8)])
def test_bond_grad_matches_ring_closed_form(T, h):
    N = 9
    lat = L.ring(N)
    g, gp = _split(lat)
    got = grad.bond_grad(g, gp, -N, N, [T], [h])[:, 0, 0]
    # every bond of the uniform ring is equivalent: d log Z / dJ (all bonds) / N
    with mp.workdps(40):
        ref = float(mp.diff(lambda J: closed_forms.ring_logz(N, T, h, J), 1)) / N
    np.testing.assert_allclose(got, ref, rtol=1e-12)


@pytest.mark.parametrize("T", [1.0, 2.269, 3.5])
def test_bond_correlation_matches_kaufman(T):
    lat = L.square_torus(4, 4)
    g, gp = _split(lat)
    got = grad.bond_correlations(g, gp, -32, 16, [T], [0.0])[:, 0, 0]
    # log Z depends on J only through J / T: log Z(J) = kaufman(T / J)
    with mp.workdps(40):
        dlogz_dJ = float(mp.diff(lambda J: closed_forms.kaufman_logz(4, 4, T / J), 1))
    np.testing.assert_allclose(got, T * dlogz_dJ / lat.n_bonds, rtol=1e-12)


def test_log_z_derivatives_match_ring_closed_form():
    N = 9
    lat = L.ring(N)
    g = native.count_all(N, lat.bond_i, lat.bond_j, lat.bond_J)
    for T, h in [(0.8, 0.0), (1.7, 0.4), (3.0, -1.0)]:
        d = grad.log_z_derivatives(g, -N, N, [T], [h])
        f = lambda t, hh: closed_forms.ring_logz(N, t, hh)   # noqa: E731
        with mp.workdps(40):
            ref = {"d_T": mp.diff(f, (T, h), (1, 0)), "d_h": mp.diff(f, (T, h), (0, 1)),
                   "d_TT": mp.diff(f, (T, h), (2, 0)), "d_Th": mp.diff(f, (T, h), (1, 1)),
                   "d_hh": mp.diff(f, (T, h), (0, 2))}
        for k, v in ref.items():
            np.testing.assert_allclose(d[k][0, 0], float(v), rtol=1e-10, atol=1e-12, err_msg=k)


def test_log_z_derivatives_match_kaufman():
    lat = L.square_torus(4, 4)
    g = native.count_all(16, lat.bond_i, lat.bond_j, lat.bond_J)
    for T in (1.2, 2.269, 4.0):
        d = grad.log_z_derivatives(g, -32, 16, [T], [0.0])
        with mp.workdps(40):
            f = lambda t: closed_forms.kaufman_logz(4, 4, t)   # noqa: E731
            np.testing.assert_allclose(d["d_T"][0, 0], float(mp.diff(f, T, 1)), rtol=1e-11)
            np.testing.assert_allclose(d["d_TT"][0, 0], float(mp.diff(f, T, 2)), rtol=1e-10)
        assert d["d_h"][0, 0] == pytest.approx(0.0, abs=1e-14)   # <M> = 0 at h = 0


# --------------------------------------------------------------------------
# non-integer couplings and per-configuration weights
# --------------------------------------------------------------------------

def test_shifted_log_z_matches_enumeration_with_real_coupling():
    lat = L.random_bond_lattice(8, 16, 9, values=(-2, -1, 1, 2))
    g, gp = _split(lat)
    s = _numpy_configs(8)
    sigma = s[:, lat.bond_i] * s[:, lat.bond_j]
    M = s.sum(axis=1)
    T, h = 1.3, 0.25
    for b in (0, 5, 11):
        for delta in (0.37, -1e-3):
            J = lat.bond_J.astype(np.float64).copy()
            J[b] += delta
            H = -(sigma * J).sum(axis=1) - h * M
            x = -H / T
            ref = x.max() + np.log(np.exp(x - x.max()).sum())
            got = grad.log_z_shifted(g, gp[b], -lat.abs_coupling_sum, 8, T, h, delta)
            assert got == pytest.approx(ref, rel=1e-13)
    lz0 = grad.log_z_shifted(g, gp[0], -lat.abs_coupling_sum, 8, T, h, 0.0)
    assert lz0 == pytest.approx(thermo.log_z(g, -lat.abs_coupling_sum, 8, [T], [h])[0, 0], rel=1e-14)


def test_bin_weights_reproduce_bond_grad_by_enumeration():
    lat = L.random_bond_lattice(9, 18, 4, values=(-1, 1, 2, 3))
    g, gp = _split(lat)
    S, N = lat.abs_coupling_sum, 9
    T = np.array([0.9, 2.0, 3.3])
    h = np.array([-0.4, 0.0, 0.6])
    G = np.random.default_rng(2).standard_normal((3, 3))
    W = grad.bin_weights(g, -S, N, T, h, G)
    # the loss gradient from the definition, configuration by configuration
    s = _numpy_configs(N)
    sigma = s[:, lat.bond_i] * s[:, lat.bond_j]
    E = -(sigma * lat.bond_J).sum(axis=1)
    nup = (s > 0).sum(axis=1)
    per_conf = W[E + S, nup]
    by_enum = (per_conf[:, None] * sigma).sum(axis=0)
    np.testing.assert_allclose(grad.bond_grad_from_weights(g, gp, W), by_enum, rtol=1e-12, atol=1e-15)
    # and from the averages: sum_{a,c} G <s_i s_j> / T
    ref = (G[None] * grad.bond_grad(g, gp, -S, N, T, h)).sum(axis=(1, 2))
    np.testing.assert_allclose(by_enum, ref, rtol=1e-11, atol=1e-14)


def test_sum_rule_bonds_times_couplings_is_mean_energy():
    lat = L.random_bond_lattice(10, 24, 3, values=(-2, -1, 1, 2))
    g, gp = _split(lat)
    S, N = lat.abs_coupling_sum, 10
    T, h = [0.8, 2.5], [0.0, 0.7]
    dJ = grad.bond_grad(g, gp, -S, N, T, h)
    mE, _, _, _ = thermo.moments(g, -S, N, T, h)
    lhs = (lat.bond_J[:, None, None] * dJ).sum(axis=0)
    np.testing.assert_allclose(lhs, -mE / np.array(T)[:, None], rtol=1e-12)


# --------------------------------------------------------------------------
# planted mistakes: the pins above must notice them
# --------------------------------------------------------------------------

def test_planted_sign_flip_breaks_kaufman_correlation_pin():
    lat = L.square_torus(4, 4)
    g, gp = _split(lat)
    T = 2.0
    wrong = grad.bond_correlations(g, g[None] - gp, -32, 16, [T], [0.0])[:, 0, 0]   # counts disagreeing spins
    with mp.workdps(30):
        ref = T * float(mp.diff(lambda J: closed_forms.kaufman_logz(4, 4, T / J), 1)) / lat.n_bonds
    assert not np.allclose(wrong, ref, rtol=1e-6)


def test_planted_missing_temperature_factor_breaks_ring_pin():
    N, T = 9, 1.5
    lat = L.ring(N)
    g, gp = _split(lat)
    wrong = grad.bond_correlations(g, gp, -N, N, [T], [0.0])[:, 0, 0]   # <s s> without the 1/T
    with mp.workdps(30):
        ref = float(mp.diff(lambda J: closed_forms.ring_logz(N, T, 0.0, J), 1)) / N
    assert not np.allclose(wrong, ref, rtol=1e-6)


def test_planted_dropped_bond_breaks_energy_identity():
    lat = L.random_bond_lattice(10, 24, 3, values=(-2, -1, 1, 2))
    g, gp = _split(lat)
    S = lat.abs_coupling_sum
    sig = 2 * gp.astype(object) - g.astype(object)[None]
    lhs = sum(int(J) * sig[b] for b, J in enumerate(lat.bond_J) if b != 4)
    E = np.arange(-S, S + 1, dtype=object)[:, None]
    assert not np.array_equal(lhs, -E * g.astype(object))


@pytest.mark.parametrize("lat", [L.square_torus(4, 5, L.pm_couplings(40, 5)),
                                 L.square_torus(5, 3, L.choice_couplings(30, 3)),
                                 L.square_torus(3, 3)], ids=lambda l: "x".join(map(str, l.dims)))
def test_transfer_matrix_bond_split_matches_brute_force(lat):
    # The shifted-coupling transfer matrix (for tori too large to enumerate on
    # the CPU) gives every bond's split table exactly as the brute force does.
    g, gp = _split(lat)
    Jh, Jv = L.torus_coupling_grids(lat)
    Lx = lat.dims[0]
    for b in range(lat.n_bonds):
        u, d = divmod(b, 2)
        g2, gp2 = native.tm_torus_bond_split(Jh, Jv, d, u % Lx, u // Lx)
        np.testing.assert_array_equal(g2, g)
        np.testing.assert_array_equal(gp2, gp[b], err_msg=f"bond {b}")
