"""Host code under sanitizers (CPU only, no GPU).

The oracle's C counts (pthreads) run under AddressSanitizer + UBSan and under
ThreadSanitizer, and the library's host-side planner (plan.cpp,
bond_plan.cpp) under AddressSanitizer + UBSan (with leak checking), each from
a small driver in tests/sanitize/.  Their outputs must match the unsanitized
oracle and library, and the sanitizers must stay silent.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import native
from paper_1110_2561_amd import api
from paper_1110_2561_amd import lattice as L

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1110_2561_amd", "csrc")


def _compile(cmd, tmp_path):
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=tmp_path)
    if r.returncode != 0:
        if "sanitizer" in (r.stderr or "").lower() or "asan" in (r.stderr or "").lower():
            pytest.skip("sanitizer runtime not available: " + r.stderr[-200:])
        raise AssertionError(r.stderr)


def _run(exe, text, env=None):
    e = dict(os.environ)
    e.update(env or {})
    r = subprocess.run([exe], input=text, capture_output=True, text=True, env=e, timeout=300)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
    assert "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-2000:]
    return r.stdout


def _lattice_text(lat):
    lines = [f"{lat.n_spins} {lat.n_bonds}"]
    lines += [f"{i} {j} {J}" for i, j, J in zip(lat.bond_i, lat.bond_j, lat.bond_J)]
    return "\n".join(lines) + "\n"


SMALL = [
    L.square_torus(3, 3),
    L.random_bond_lattice(10, 25, 2, values=(-2, -1, 1, 2)),
    L.Lattice(5, [0, 0, 1, 3], [1, 1, 2, 4], [2, -2, 1, 3]),      # a pair whose couplings cancel
    L.ring(7, L.pm_couplings(7, 4)),
]


def _oracle_expected(lat):
    g, gp = native.bond_split(lat.n_spins, lat.bond_i, lat.bond_j, lat.bond_J)
    S = lat.abs_coupling_sum
    lines = [f"{e - S} {u} {int(g[e, u])}" for e, u in zip(*np.nonzero(g))]
    lines.append("split")
    for b in range(lat.n_bonds):
        lines += [f"bond {b} {e - S} {u} {int(gp[b, e, u])}" for e, u in zip(*np.nonzero(gp[b]))]
    return lines


@pytest.mark.parametrize("flags,env", [
    (["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"], {"ASAN_OPTIONS": "detect_leaks=1"}),
    (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}),
], ids=["asan-ubsan", "tsan"])
def test_oracle_under_sanitizers(tmp_path, flags, env):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_driver")
    _compile(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", *flags, "-pthread",
              os.path.join(HERE, "sanitize", "oracle_driver.c"), os.path.join(ROOT, "oracle", "oracle.c"),
              "-o", exe], tmp_path)
    for lat in SMALL:
        out = _run(exe, _lattice_text(lat), env).strip().splitlines()
        assert out == _oracle_expected(lat), lat.kind


PLAN_LATTICES = SMALL + [
    L.Lattice(1, [], [], []),
    L.square_torus(6, 6),
    L.square_torus(8, 5, L.pm_couplings(80, 20111025)),
    L.square_torus(8, 8, L.pm_couplings(128, 64)),                    # N = 64
    L.cubic_torus(4, L.choice_couplings(192, 4)),                      # N = 64, wide energy range
    L.triangular_free(31, 6, L.choice_couplings(L.triangular_free(31, 6).n_bonds, 9)),
    L.random_bond_lattice(40, 300, 3, values=(-3, -2, -1, 1, 2, 3, 4, 5)),   # 8 coupling classes
    L.Lattice(3, [0, 0], [0, 1], [1, 1]),                              # a self-bond: rejected
    L.Lattice(4, [0], [7], [1]),                                       # endpoint out of range
]
TUNES = [api.Tune(), api.Tune(tile_bits=3, waves_per_block=4), api.Tune(replicas=4), api.Tune(prefix_bits=5),
         api.Tune(inner_bits=12, tile_bits=8)]


def _plan_expected(lat, idx):
    lines = []
    for t, tune in enumerate(TUNES):
        head = f"lattice {idx} tune {t}"
        try:
            p = api.Plan(lat, tune)
        except api.IsingError as e:
            lines.append(f"{head} status {e.code}")
            continue
        try:
            ws = p.bond_workspace_bytes
            wst = 0
        except api.IsingError as e:
            ws, wst = 0, e.code
        bits = " ".join(str(int(b)) for b in p.bit_of_site)
        lines.append(f"{head} status 0 shape {p.n_e} {p.n_m} {p.e_min} inner {p.inner_bits} tile {p.tile_bits} "
                     f"chunks {p.n_chunks} ws {wst} {ws} bits {bits}")
        p.close()
    return lines


def test_planner_under_asan_ubsan(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "plan_driver")
    _compile(["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
              "-fno-sanitize-recover=undefined", "-I", os.path.join(ROOT, "include"),
              os.path.join(HERE, "sanitize", "plan_driver.cpp"), os.path.join(CSRC, "plan.cpp"),
              os.path.join(CSRC, "bond_plan.cpp"), "-o", exe], tmp_path)
    text = "".join(_lattice_text(lat) for lat in PLAN_LATTICES)
    out = _run(exe, text, {"ASAN_OPTIONS": "detect_leaks=1"}).strip().splitlines()
    expected = []
    for idx, lat in enumerate(PLAN_LATTICES):
        expected += _plan_expected(lat, idx)
    assert out == expected
