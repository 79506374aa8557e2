"""Checkpointed, resumable enumeration (paper_1110_2561_amd.checkpoint), on the
CPU: the runner's host logic with the oracle's brute force standing in for
the GPU range call (the test supplies it; the library never does).  A run cut
short - by a piece limit, or by killing its process in the middle of a piece -
resumes from the last checkpoint to exactly the uninterrupted table."""
import os
import subprocess
import sys
import textwrap

import numpy as np
import pytest

from oracle import native
from paper_1110_2561_amd import api, checkpoint
from paper_1110_2561_amd import lattice as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LAT = L.square_torus(4, 5, L.pm_couplings(40, 5))
TUNE = api.Tune(inner_bits=12)


def oracle_range(plan):
    """Adds the brute-force counts of a chunk range (the plan's bit order) to a CPU table."""
    rel = plan.lattice.relabel(plan.bit_of_site)
    k = plan.inner_bits

    def add(first, n, g):
        g.numpy()[...] += native.count_range(rel.n_spins, rel.bond_i, rel.bond_j, rel.bond_J,
                                             first << k, n << k, n_threads=2)
    return add


def whole():
    return native.count_all(LAT.n_spins, LAT.bond_i, LAT.bond_j, LAT.bond_J)


def test_pieces_and_resume_equal_the_whole(tmp_path):
    plan = api.Plan(LAT, TUNE)
    assert plan.n_chunks == 256
    path = str(tmp_path / "run.npz")
    g, done = checkpoint.run(plan, path, piece_chunks=37, max_pieces=3, range_fn=oracle_range(plan), device="cpu")
    assert not done
    table, nxt = checkpoint.load(path, plan)
    assert nxt == 3 * 37 and np.array_equal(table, g.numpy())
    plan2 = api.Plan(LAT, TUNE)                      # a fresh process would build the same plan
    g2, done = checkpoint.run(plan2, path, piece_chunks=50, range_fn=oracle_range(plan2), device="cpu")
    assert done
    np.testing.assert_array_equal(g2.numpy(), whole())
    # a finished checkpoint resumes to the same table with no further work
    g3, done = checkpoint.run(plan2, path, range_fn=lambda *a: pytest.fail("no work left"), device="cpu")
    assert done and np.array_equal(g3.numpy(), g2.numpy())


def test_killed_run_resumes(tmp_path):
    path = str(tmp_path / "run.npz")
    script = textwrap.dedent(f"""
        import os, sys
        sys.path.insert(0, {ROOT!r})
        sys.path.insert(0, {os.path.join(ROOT, 'tests')!r})
        from test_checkpoint import LAT, TUNE, oracle_range
        from paper_1110_2561_amd import api, checkpoint
        plan = api.Plan(LAT, TUNE)
        add = oracle_range(plan)
        calls = [0]
        def dying(first, n, g):
            calls[0] += 1
            if calls[0] == 4:
                add(first, n // 2, g)      # half of the piece is counted, then the process dies
                os._exit(3)
            add(first, n, g)
        checkpoint.run(plan, {path!r}, piece_chunks=20, range_fn=dying, device="cpu")
    """)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=300)
    assert r.returncode == 3, r.stderr[-2000:]
    plan = api.Plan(LAT, TUNE)
    table, nxt = checkpoint.load(path, plan)
    assert nxt == 60                                  # three whole pieces were saved
    g, done = checkpoint.run(plan, path, piece_chunks=64, range_fn=oracle_range(plan), device="cpu")
    assert done
    np.testing.assert_array_equal(g.numpy(), whole())


def test_checkpoint_of_another_plan_is_refused(tmp_path):
    path = str(tmp_path / "run.npz")
    plan = api.Plan(LAT, TUNE)
    checkpoint.run(plan, path, piece_chunks=16, max_pieces=1, range_fn=oracle_range(plan), device="cpu")
    other_couplings = api.Plan(L.square_torus(4, 5, L.pm_couplings(40, 6)), TUNE)
    other_layout = api.Plan(LAT, api.Tune(inner_bits=10))
    for p in (other_couplings, other_layout):
        with pytest.raises(ValueError):
            checkpoint.load(path, p)
        with pytest.raises(ValueError):
            checkpoint.run(p, path, range_fn=oracle_range(p), device="cpu")


def test_save_rejects_bad_state(tmp_path):
    plan = api.Plan(LAT, TUNE)
    path = str(tmp_path / "run.npz")
    with pytest.raises(ValueError):
        checkpoint.save(path, plan, np.zeros((3, 3), dtype=np.uint64), 0)
    with pytest.raises(ValueError):
        checkpoint.save(path, plan, np.zeros((plan.n_e, plan.n_m), dtype=np.uint64), plan.n_chunks + 1)
    assert not os.path.exists(path)
