"""log Z(T, h, J) as a differentiable PyTorch function.

The forward is Eq. (2) of Peretyatko et al. evaluated from the exact table
g(E, M) (enumerated once per lattice).  The backward is written by hand from
the derivatives of that sum, with H = E - h M and E = -sum_b J_b s_i s_j:
  d log Z / dT   = <H>/T^2,   d log Z / dh = <M>/T      (from g, FP64),
  d log Z / dJ_b = <s_i s_j>/T                          (recomputed enumeration:
      the loss gradient G[T][h] becomes a per-bin weight W(E, M), and one more
      pass over all configurations sums W s_i s_j per bond in FP64).
The (T, h) gradient is itself differentiable (second derivatives from g), so
a double backward gives the heat capacity and susceptibility:
  C = d<H>/dT with <H> = T^2 d log Z/dT,  chi = d<M>/dh with <M> = T d log Z/dh.
Second derivatives that involve J are not provided (they raise).

The couplings J must hold the lattice's integer values: the enumeration is
exact for those, and J is an input only so that gradients can flow to it.
"""
from __future__ import annotations

import numpy as np
import torch

from . import api
from .lattice import Lattice

__all__ = ["IsingLogZ", "log_z"]


class _NotTwiceDifferentiable(torch.autograd.Function):
    """Passes the coupling gradient through, attached to the graph of its
    inputs, so that differentiating it again raises instead of giving 0."""

    @staticmethod
    def forward(ctx, x, *inputs):
        return x.clone()

    @staticmethod
    def backward(ctx, g):
        raise RuntimeError("second derivatives of log Z that involve the couplings J are not implemented")


class _LogZFirst(torch.autograd.Function):
    """(d log Z/dT, d log Z/dh) on the grid; its backward uses the second derivatives."""

    @staticmethod
    def forward(ctx, T, h, model):
        d = api.logz_derivatives(model.g, model.plan.e_min, model.plan.n_spins, T.detach(), h.detach())
        ctx.save_for_backward(d["d_TT"], d["d_Th"], d["d_hh"])
        return d["d_T"], d["d_h"]

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, g_dT, g_dh):
        d_TT, d_Th, d_hh = ctx.saved_tensors
        g_dT = torch.zeros_like(d_TT) if g_dT is None else g_dT
        g_dh = torch.zeros_like(d_TT) if g_dh is None else g_dh
        gT = (g_dT * d_TT + g_dh * d_Th).sum(dim=1)
        gh = (g_dT * d_Th + g_dh * d_hh).sum(dim=0)
        return gT, gh, None


class _LogZ(torch.autograd.Function):
    @staticmethod
    def forward(ctx, T, h, J, model):
        lz = api.log_z(model.g, model.plan.e_min, model.plan.n_spins, T.detach(), h.detach())
        ctx.model = model
        ctx.save_for_backward(T, h, J, lz)
        return lz

    @staticmethod
    def backward(ctx, go):
        T, h, J, lz = ctx.saved_tensors
        model = ctx.model
        go = go.to(torch.float64).contiguous()
        need = ctx.needs_input_grad[:3]
        if not torch.is_grad_enabled():
            # no graph to build: the whole backward in one library call
            gT, gh, gJ = api.logz_backward(model.plan, model.g, T.detach(), h.detach(), lz, go, want=need,
                                           symmetric=model.symmetric_backward)
            return gT, gh, gJ, None
        gT = gh = gJ = None
        if need[0] or need[1]:
            # building a graph for a double backward: the first derivatives as
            # a differentiable function of (T, h)
            dT, dh = _LogZFirst.apply(T, h, model)
            gT = (go * dT).sum(dim=1) if need[0] else None
            gh = (go * dh).sum(dim=0) if need[1] else None
        if need[2]:
            # the weight table is only read by the backward kernel that follows
            # on the same stream, so the model's buffer is reused call to call
            W = api.bin_weights(model.g, model.plan.e_min, model.plan.n_spins, T.detach(), h.detach(), lz,
                                go.detach(), out=model.weights_buffer())
            gJ = api.bond_backward(model.plan, W, symmetric=model.symmetric_backward)
            if torch.is_grad_enabled():
                gJ = _NotTwiceDifferentiable.apply(gJ, T, h, J)
        return gT, gh, gJ, None


class IsingLogZ:
    """log Z(T, h, J) of one lattice: enumerates g(E, M) once, then evaluates
    and differentiates Eq. (2) on any (T, h) grid.

    __call__(T [nT], h [nh], J [n_bonds] or None) -> log Z [nT, nh] (float64, on the GPU);
    T and h are cast to float64 (differentiably).  With symmetric_backward the
    per-bond gradient walks half of the configurations (spin-flip symmetry,
    api.bond_backward(symmetric=True)); the default recomputes all of them.

    Backward passes of one instance reuse its weight buffer and the plan's
    workspace in stream order: backward passes that overlap in time on
    different streams need instances of their own.
    """

    def __init__(self, lattice: Lattice, tune: api.Tune | None = None, symmetric_backward: bool = False):
        self.lattice = lattice
        self.symmetric_backward = bool(symmetric_backward)
        self.plan = api.Plan(lattice, tune)
        self.g = api.enumerate_g(self.plan)
        self._J = np.asarray(lattice.bond_J, dtype=np.float64)
        self._J_dev = torch.as_tensor(self._J, dtype=torch.float64, device=self.g.device)
        self._W = None
        # (tensor, version counter) of the coupling tensor last checked against
        # the lattice: checking costs a device-to-host copy, so a tensor is
        # checked again only after an in-place change
        self._checked = None

    def couplings(self, device="cuda", requires_grad: bool = True) -> torch.Tensor:
        return torch.tensor(self._J, dtype=torch.float64, device=device, requires_grad=requires_grad)

    def weights_buffer(self) -> torch.Tensor:
        """[n_e][n_m] FP64 device buffer for the backward's bin weights."""
        if self._W is None:
            self._W = torch.empty((self.plan.n_e, self.plan.n_m), dtype=torch.float64, device=self.g.device)
        return self._W

    def _check_couplings(self, J: torch.Tensor):
        if J.shape != (self.lattice.n_bonds,) or J.dtype != torch.float64:
            raise ValueError(f"J must be a float64 tensor of shape ({self.lattice.n_bonds},)")
        seen = self._checked
        if seen is not None and seen[0] is J and seen[1] == J._version:
            return
        if not np.array_equal(J.detach().cpu().numpy(), self._J):
            raise ValueError("J must hold the lattice's integer couplings (the enumeration is exact for those)")
        self._checked = (J, J._version)

    def __call__(self, T, h, J: torch.Tensor | None = None) -> torch.Tensor:
        dev = self.g.device
        T = T if isinstance(T, torch.Tensor) else torch.as_tensor(np.atleast_1d(T), dtype=torch.float64, device=dev)
        h = h if isinstance(h, torch.Tensor) else torch.as_tensor(np.atleast_1d(h), dtype=torch.float64, device=dev)
        if T.dim() != 1 or h.dim() != 1:
            raise ValueError("T and h must be 1-D tensors")
        T, h = T.to(device=dev, dtype=torch.float64), h.to(device=dev, dtype=torch.float64)   # differentiable casts
        if J is None:
            J = self._J_dev
        else:
            self._check_couplings(J)
        return _LogZ.apply(T, h, J, self)


def log_z(lattice: Lattice, T, h, J: torch.Tensor | None = None) -> torch.Tensor:
    """One-shot differentiable log Z [nT, nh]; see IsingLogZ."""
    return IsingLogZ(lattice)(T, h, J)
