"""The table dump (paper_1110_2561_amd.table) and the command line's host
logic (lattice specs, coupling draws, grids), on the CPU."""
import io
import json

import numpy as np
import pytest
import torch

from conftest import load_table1
from oracle import native
from paper_1110_2561_amd import __main__ as cli
from paper_1110_2561_amd import lattice as L
from paper_1110_2561_amd import table


def test_rows_of_the_4x4_table_are_table1():
    lat = L.square_torus(4, 4)
    g = native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    r = table.rows(g, -32, 16)
    assert {(e, m): c for c, m, e in r} == load_table1()
    assert r == sorted(r, key=lambda x: (x[1], x[2]))
    assert sum(c for c, _, _ in r) == 1 << 16
    # a torch table (as the library returns) gives the same rows
    t = torch.from_numpy(g.view(np.int64)).view(torch.uint64)
    assert table.rows(t, -32, 16) == r


def test_write_read_round_trip(tmp_path):
    lat = L.ring(7, L.pm_couplings(7, 2))
    g = native.count_all(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    path = tmp_path / "t.txt"
    table.write(str(path), g, -lat.abs_coupling_sum, 7, header=["ring"])
    assert path.read_text().startswith("# ring\n# count M E\n")
    assert table.read(str(path)) == table.rows(g, -lat.abs_coupling_sum, 7)
    buf = io.StringIO()
    table.write(buf, g, -lat.abs_coupling_sum, 7)
    buf.seek(0)
    assert table.read(buf) == table.rows(g, -lat.abs_coupling_sum, 7)
    with pytest.raises(ValueError):
        table.rows(g, -lat.abs_coupling_sum, 8)


def test_lattice_specs(tmp_path):
    assert cli.parse_lattice("torus:4x5").n_spins == 20 and cli.parse_lattice("torus:4x5").n_bonds == 40
    assert cli.parse_lattice("ring:9").n_bonds == 9
    assert cli.parse_lattice("cubic:3").n_bonds == 81
    tri = cli.parse_lattice("triangular:19x5")
    assert tri.n_spins == 19 and tri.n_bonds == L.triangular_free(19, 5).n_bonds
    lat = L.square_torus(3, 4, L.pm_couplings(24, 7), seed=7)
    path = tmp_path / "l.json"
    path.write_text(lat.to_json())
    back = cli.parse_lattice(str(path))
    np.testing.assert_array_equal(back.bond_J, lat.bond_J)
    with pytest.raises(SystemExit):
        cli.parse_lattice("torus:4by5")


def test_coupling_draws_and_grids():
    lat = L.square_torus(8, 5)
    pm = cli.with_couplings(lat, 20111025, None)
    np.testing.assert_array_equal(pm.bond_J, L.workload("torus8x5_pm")["lattice"].bond_J)
    ch = cli.with_couplings(lat, None, "3:-2,-1,1,2")
    np.testing.assert_array_equal(ch.bond_J, L.choice_couplings(80, 3, (-2, -1, 1, 2)))
    assert cli.with_couplings(lat, None, None) is lat
    np.testing.assert_allclose(cli.parse_grid("0.5:5:4"), [0.5, 2.0, 3.5, 5.0])
    np.testing.assert_allclose(cli.parse_grid("0,0.1"), [0.0, 0.1])
