"""Python front end over libising: plans, enumeration, log Z and moments.

PyTorch provides device memory and the current HIP stream; every step of the
computation runs in the library's kernels (there is no CPU fallback).
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib
from .lattice import Lattice

__all__ = ["Plan", "Tune", "enumerate_g", "enumerate_range", "log_z", "moments", "IsingError"]

IsingError = _lib.IsingError


@dataclass
class Tune:
    inner_bits: int = 0
    tile_bits: int = 0
    waves_per_block: int = 0
    replicas: int = 0
    max_blocks: int = 0

    def _c(self):
        return _lib.ising_tune(self.inner_bits, self.tile_bits, self.waves_per_block, self.replicas,
                               self.max_blocks)


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


class Plan:
    """An immutable enumeration plan for one lattice (ising_plan_create)."""

    def __init__(self, lattice: Lattice, tune: Tune | None = None):
        self.lattice = lattice
        bi = np.ascontiguousarray(lattice.bond_i, dtype=np.int32)
        bj = np.ascontiguousarray(lattice.bond_j, dtype=np.int32)
        bJ = np.ascontiguousarray(lattice.bond_J, dtype=np.int32)
        p = _lib.i32p
        lat = _lib.ising_lattice(int(lattice.n_spins), int(bi.shape[0]), bi.ctypes.data_as(p),
                                 bj.ctypes.data_as(p), bJ.ctypes.data_as(p))
        handle = ctypes.c_void_p()
        tn = tune._c() if tune is not None else None
        _lib.check(_lib.ising_plan_create(ctypes.byref(lat), ctypes.byref(tn) if tn is not None else None,
                                          ctypes.byref(handle)))
        self._h = handle
        n_e, n_m, e_min = _lib.i32(), _lib.i32(), _lib.i32()
        _lib.check(_lib.ising_hist_shape(self._h, ctypes.byref(n_e), ctypes.byref(n_m), ctypes.byref(e_min)))
        self.n_e, self.n_m, self.e_min = n_e.value, n_m.value, e_min.value
        bos = (ctypes.c_int32 * lattice.n_spins)()
        k, j, nc = _lib.i32(), _lib.i32(), _lib.u64()
        _lib.check(_lib.ising_plan_layout(self._h, bos, ctypes.byref(k), ctypes.byref(j), ctypes.byref(nc)))
        self.bit_of_site = np.array(bos[:], dtype=np.int64)
        self.inner_bits, self.tile_bits, self.n_chunks = k.value, j.value, nc.value

    @property
    def n_spins(self) -> int:
        return self.lattice.n_spins

    @property
    def handle(self):
        return self._h

    def new_table(self, device="cuda") -> torch.Tensor:
        return torch.empty((self.n_e, self.n_m), dtype=torch.uint64, device=device)

    def close(self):
        if getattr(self, "_h", None):
            _lib.ising_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_table(plan: Plan, g: torch.Tensor):
    if not (g.is_cuda and g.dtype == torch.uint64 and g.is_contiguous()
            and tuple(g.shape) == (plan.n_e, plan.n_m)):
        raise ValueError(f"g must be a contiguous CUDA uint64 tensor of shape {(plan.n_e, plan.n_m)}")


def enumerate_g(plan: Plan, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """g(E, M) of all configurations (ising_enumerate)."""
    g = plan.new_table() if out is None else out
    _check_table(plan, g)
    _lib.check(_lib.ising_enumerate(plan.handle, g.data_ptr(), _stream_handle(stream)))
    return g


def enumerate_range(plan: Plan, first_chunk: int, n_chunks: int, g: torch.Tensor, stream=None) -> torch.Tensor:
    """Add the counts of chunks [first_chunk, first_chunk + n_chunks) to g."""
    _check_table(plan, g)
    _lib.check(_lib.ising_enumerate_range(plan.handle, int(first_chunk), int(n_chunks), g.data_ptr(),
                                          _stream_handle(stream)))
    return g


def _grid(x, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).reshape(-1).contiguous()
    return torch.as_tensor(np.atleast_1d(np.asarray(x, dtype=np.float64)), device=device).contiguous()


def log_z(g: torch.Tensor, e_min: int, n_spins: int, T, h, stream=None) -> torch.Tensor:
    """log Z [len(T), len(h)] in FP64 from a dense device table (ising_logz)."""
    Tt, ht = _grid(T, g.device), _grid(h, g.device)
    out = torch.empty((Tt.numel(), ht.numel()), dtype=torch.float64, device=g.device)
    n_e, n_m = g.shape
    _lib.check(_lib.ising_logz(g.data_ptr(), n_e, n_m, int(e_min), int(n_spins), Tt.data_ptr(), Tt.numel(),
                               ht.data_ptr(), ht.numel(), out.data_ptr(), _stream_handle(stream)))
    return out


def moments(g: torch.Tensor, e_min: int, n_spins: int, T, h, stream=None) -> dict:
    """log Z, <E>, <M>, C = Var(E - hM)/T^2, chi = Var(M)/T, each [len(T), len(h)]."""
    Tt, ht = _grid(T, g.device), _grid(h, g.device)
    shape = (Tt.numel(), ht.numel())
    outs = {k: torch.empty(shape, dtype=torch.float64, device=g.device)
            for k in ("log_z", "mean_E", "mean_M", "heat_capacity", "susceptibility")}
    n_e, n_m = g.shape
    _lib.check(_lib.ising_moments(g.data_ptr(), n_e, n_m, int(e_min), int(n_spins), Tt.data_ptr(), Tt.numel(),
                                  ht.data_ptr(), ht.numel(), outs["log_z"].data_ptr(), outs["mean_E"].data_ptr(),
                                  outs["mean_M"].data_ptr(), outs["heat_capacity"].data_ptr(),
                                  outs["susceptibility"].data_ptr(), _stream_handle(stream)))
    return outs
