"""The allocation-free per-bond backward, ising_bond_backward_noalloc,
against ising_bond_backward (workspace form) through the C ABI: two calls in
a row on one device, the second with a smaller lattice, each equal to the
workspace form bit for bit (same kernels, same summation order); a plan whose
tables are not yet on the device is refused instead of uploaded."""
import numpy as np
import pytest
import torch

from paper_1110_2561_amd import lattice as L

pytestmark = pytest.mark.gpu


def _weights(g_shape, seed):
    rng = np.random.default_rng(seed)
    W = rng.standard_normal(g_shape) * np.exp(-rng.uniform(0, 3, g_shape))
    return torch.from_numpy(W).cuda()


def test_noalloc_backward_equals_workspace_form_twice():
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    from paper_1110_2561_amd import _lib, api
    stream = torch.cuda.current_stream().cuda_stream or None
    big = L.cubic_torus(3, L.choice_couplings(81, 6))                  # 27 spins, 81 bonds, 4 couplings
    small = L.square_torus(4, 5, L.pm_couplings(40, 5))              # 20 spins, 40 bonds
    for k, lat in enumerate((big, small)):
        plan = api.Plan(lat)
        W = _weights((plan.n_e, plan.n_m), 10 + k)
        print(f"call {k}: N={lat.n_spins} bonds={lat.n_bonds}", flush=True)
        if k == 0:
            # nothing uploaded yet on this device: refused, nothing launched
            out = torch.full((lat.n_bonds,), float("nan"), dtype=torch.float64, device="cuda")
            rc = _lib.ising_bond_backward_noalloc(plan.handle, W.data_ptr(), out.data_ptr(), stream)
            assert rc == -1 and "not on device" in _lib.ising_last_error().decode()
        ref = api.bond_backward(plan, W)                                 # uploads the tables
        out = torch.full((lat.n_bonds,), float("nan"), dtype=torch.float64, device="cuda")
        _lib.check(_lib.ising_bond_backward_noalloc(plan.handle, W.data_ptr(), out.data_ptr(), stream))
        torch.cuda.synchronize()
        assert torch.equal(out, ref), k


def test_noalloc_argument_errors():
    from paper_1110_2561_amd import _lib, api
    plan = api.Plan(L.ring(6))
    W = torch.zeros((plan.n_e, plan.n_m), dtype=torch.float64, device="cuda")
    api.bond_backward(plan, W)
    out = torch.zeros(6, dtype=torch.float64, device="cuda")
    assert _lib.ising_bond_backward_noalloc(None, W.data_ptr(), out.data_ptr(), None) == -1
    assert _lib.ising_bond_backward_noalloc(plan.handle, None, out.data_ptr(), None) == -1
    assert _lib.ising_bond_backward_noalloc(plan.handle, W.data_ptr(), None, None) == -1
    torch.cuda.synchronize()
