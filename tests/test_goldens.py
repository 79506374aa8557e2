"""The stored oracle tables of the batch256 cubes (tests/golden/batch256_cubes.npz,
written by tests/golden/make_batch256_cubes.py with the oracle's brute force):
they cover every cube of the workload, satisfy the invariants of any table
(Section 2: sum g = 2^N, binomial marginals; g(E, M) = g(E, -M)), and two of
them, re-counted now by the same brute force, are unchanged."""
import numpy as np
import pytest

from conftest import load_cube_goldens
from oracle import closed_forms, native
from paper_1110_2561_amd import lattice as L


@pytest.fixture(scope="module")
def cubes():
    return load_cube_goldens()


def test_goldens_cover_every_cube(cubes):
    lats = L.workload("batch256")["lattices"]
    assert sorted(cubes) == [i for i, lat in enumerate(lats) if lat.kind == "cubic_torus"]
    assert len(cubes) == 85


def test_goldens_satisfy_table_invariants(cubes):
    lats = L.workload("batch256")["lattices"]
    marg = closed_forms.binomial_marginal(27)
    for i, g in cubes.items():
        S = lats[i].abs_coupling_sum
        assert g.shape == (2 * S + 1, 28), i
        assert int(g.sum()) == 1 << 27, i
        np.testing.assert_array_equal(g.sum(axis=0).astype(object), marg)
        np.testing.assert_array_equal(g, g[:, ::-1])


@pytest.mark.slow
def test_goldens_recount(cubes):
    lats = L.workload("batch256")["lattices"]
    members = sorted(cubes)
    for i in (members[0], members[-1]):
        lat = lats[i]
        np.testing.assert_array_equal(native.count_all(27, lat.bond_i, lat.bond_j, lat.bond_J), cubes[i])
