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

__all__ = ["Plan", "Tune", "enumerate_g", "enumerate_symmetric", "enumerate_range", "log_z", "moments",
           "IsingError",
           "logz_derivatives", "bin_weights", "bond_backward", "logz_backward",
           "BatchPlan", "batch_enumerate", "batch_moments", "BatchGraph"]

IsingError = _lib.IsingError


@dataclass
class Tune:
    inner_bits: int = 0
    tile_bits: int = 0
    waves_per_block: int = 0
    replicas: int = 0
    max_blocks: int = 0
    prefix_bits: int = 0

    def _c(self):
        return _lib.ising_tune(self.inner_bits, self.tile_bits, self.waves_per_block, self.replicas,
                               self.max_blocks, self.prefix_bits)


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

    @property
    def bond_workspace_bytes(self) -> int:
        """Device workspace of bond_backward (ising_bond_workspace); raises
        IsingError when the per-bond backward does not support this lattice.
        A plan is immutable, so the size is asked for once."""
        if getattr(self, "_bw_bytes", None) is None:
            n = ctypes.c_size_t()
            _lib.check(_lib.ising_bond_workspace(self._h, ctypes.byref(n)))
            self._bw_bytes = n.value
        return self._bw_bytes

    def bond_workspace(self, device) -> torch.Tensor:
        """The plan's backward workspace on `device`, allocated on first use and
        kept.  Calls that use it are stream-ordered; calls on different streams
        that overlap in time must pass workspaces of their own."""
        device = torch.device(device)
        cache = self.__dict__.setdefault("_ws", {})
        ws = cache.get(device)
        if ws is None:
            ws = torch.empty(max(self.bond_workspace_bytes, 8), dtype=torch.uint8, device=device)
            cache[device] = ws
        return ws

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


def enumerate_symmetric(plan: Plan, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """g(E, M) from the half of the configurations with the top plan bit up,
    mirrored M -> -M (ising_enumerate_symmetric); equal to enumerate_g."""
    g = plan.new_table() if out is None else out
    _check_table(plan, g)
    _lib.check(_lib.ising_enumerate_symmetric(plan.handle, g.data_ptr(), _stream_handle(stream)))
    return g


def enumerate_range(plan: Plan, first_chunk: int, n_chunks: int, g: torch.Tensor, stream=None) -> torch.Tensor:
    """Add the counts of chunks [first_chunk, first_chunk + n_chunks) to g."""
    _check_table(plan, g)
    _lib.check(_lib.ising_enumerate_range(plan.handle, int(first_chunk), int(n_chunks), g.data_ptr(),
                                          _stream_handle(stream)))
    return g


def _check_dense(g: torch.Tensor):
    if not (isinstance(g, torch.Tensor) and g.is_cuda and g.dtype == torch.uint64 and g.dim() == 2
            and g.is_contiguous()):
        raise ValueError("g must be a contiguous 2-D CUDA uint64 table [n_e, n_m]")


def _check_out(t: torch.Tensor, shape: tuple, device, name: str):
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float64 and t.is_contiguous()
            and tuple(t.shape) == tuple(shape) and t.device == device):
        raise ValueError(f"{name} must be a contiguous float64 tensor of shape {tuple(shape)} on {device}")


def _grid(x, device) -> torch.Tensor:
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=torch.float64).reshape(-1).contiguous()
    return torch.as_tensor(np.atleast_1d(np.asarray(x, dtype=np.float64)), device=device).contiguous()


def log_z(g: torch.Tensor, e_min: int, n_spins: int, T, h, stream=None) -> torch.Tensor:
    """log Z [len(T), len(h)] in FP64 from a dense device table (ising_logz)."""
    _check_dense(g)
    Tt, ht = _grid(T, g.device), _grid(h, g.device)
    out = torch.empty((Tt.numel(), ht.numel()), dtype=torch.float64, device=g.device)
    n_e, n_m = g.shape
    _lib.check(_lib.ising_logz(g.data_ptr(), n_e, n_m, int(e_min), int(n_spins), Tt.data_ptr(), Tt.numel(),
                               ht.data_ptr(), ht.numel(), out.data_ptr(), _stream_handle(stream)))
    return out


def moments(g: torch.Tensor, e_min: int, n_spins: int, T, h, stream=None) -> dict:
    """log Z, <E>, <M>, C = Var(E - hM)/T^2, chi = Var(M)/T, each [len(T), len(h)]."""
    _check_dense(g)
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


def logz_derivatives(g: torch.Tensor, e_min: int, n_spins: int, T, h, stream=None, second: bool = True) -> dict:
    """log Z and its first and second derivatives in (T, h), each [len(T), len(h)]
    (ising_logz_derivatives): keys log_z, d_T, d_h, d_TT, d_Th, d_hh; with
    second=False only log_z, d_T and d_h (the kernel then skips its
    second-moment pass)."""
    _check_dense(g)
    Tt, ht = _grid(T, g.device), _grid(h, g.device)
    shape = (Tt.numel(), ht.numel())
    keys = ("log_z", "d_T", "d_h", "d_TT", "d_Th", "d_hh") if second else ("log_z", "d_T", "d_h")
    outs = {k: torch.empty(shape, dtype=torch.float64, device=g.device) for k in keys}
    ptrs = [outs[k].data_ptr() if k in outs else None for k in ("log_z", "d_T", "d_h", "d_TT", "d_Th", "d_hh")]
    n_e, n_m = g.shape
    _lib.check(_lib.ising_logz_derivatives(g.data_ptr(), n_e, n_m, int(e_min), int(n_spins), Tt.data_ptr(),
                                           Tt.numel(), ht.data_ptr(), ht.numel(), *ptrs, _stream_handle(stream)))
    return outs


def bin_weights(g: torch.Tensor, e_min: int, n_spins: int, T, h, logz: torch.Tensor, grad: torch.Tensor,
                out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Per-configuration weights W[n_e, n_m] of the loss sum(grad * log Z) (ising_bin_weights)."""
    _check_dense(g)
    Tt, ht = _grid(T, g.device), _grid(h, g.device)
    shape = (Tt.numel(), ht.numel())
    lz = logz.to(device=g.device, dtype=torch.float64).contiguous()
    gr = grad.to(device=g.device, dtype=torch.float64).contiguous()
    if tuple(lz.shape) != shape or tuple(gr.shape) != shape:
        raise ValueError(f"logz and grad must have shape {shape}")
    W = torch.empty(tuple(g.shape), dtype=torch.float64, device=g.device) if out is None else out
    _check_out(W, tuple(g.shape), g.device, "out")
    n_e, n_m = g.shape
    _lib.check(_lib.ising_bin_weights(g.data_ptr(), n_e, n_m, int(e_min), int(n_spins), Tt.data_ptr(), Tt.numel(),
                                      ht.data_ptr(), ht.numel(), lz.data_ptr(), gr.data_ptr(), W.data_ptr(),
                                      _stream_handle(stream)))
    return W


def bond_backward(plan: Plan, W: torch.Tensor, out: torch.Tensor | None = None, stream=None,
                  symmetric: bool = False) -> torch.Tensor:
    """dJ[b] = sum over all configurations of W(E, M) s_i s_j per input bond (ising_bond_backward);
    with symmetric, from the half of the configurations with the top spin up and weights
    W(E, M) + W(E, -M) (ising_bond_backward_symmetric)."""
    if not (W.is_cuda and W.dtype == torch.float64 and W.is_contiguous() and tuple(W.shape) == (plan.n_e, plan.n_m)):
        raise ValueError(f"W must be a contiguous CUDA float64 tensor of shape {(plan.n_e, plan.n_m)}")
    nb = plan.lattice.n_bonds
    dJ = torch.empty(nb, dtype=torch.float64, device=W.device) if out is None else out
    _check_out(dJ, (nb,), W.device, "out")
    ws = plan.bond_workspace(W.device)
    fn = _lib.ising_bond_backward_symmetric if symmetric else _lib.ising_bond_backward
    _lib.check(fn(plan.handle, W.data_ptr(), dJ.data_ptr(), ws.data_ptr(), ws.numel(), _stream_handle(stream)))
    return dJ


def logz_backward(plan: Plan, g: torch.Tensor, T: torch.Tensor, h: torch.Tensor, logz: torch.Tensor,
                  grad: torch.Tensor, want=(True, True, True), symmetric: bool = False, stream=None):
    """(dL/dT, dL/dh, dL/dJ) of L = sum(grad * log Z) for the plan's lattice in
    one library call (ising_logz_backward); an entry is None where `want` is
    false.  T, h: 1-D float64 device tensors; logz, grad: [len(T), len(h)]
    float64 device tensors; g: the plan's table.  The workspace is kept on the
    plan, one per device (stream-ordered reuse: calls that overlap in time on
    different streams need plans of their own)."""
    _check_table(plan, g)
    dev = g.device
    Tt, ht = _grid(T, dev), _grid(h, dev)
    nT, nh = Tt.numel(), ht.numel()
    lz = logz if logz.is_contiguous() else logz.contiguous()
    G = grad if grad.is_contiguous() else grad.contiguous()
    if lz.dtype != torch.float64 or G.dtype != torch.float64 or lz.shape != (nT, nh) or G.shape != (nT, nh):
        raise ValueError(f"logz and grad must be float64 tensors of shape {(nT, nh)}")
    # one workspace per device, grown to the largest grid seen (the size of
    # each grid shape is asked for once)
    sizes = plan.__dict__.setdefault("_lb_bytes", {})
    need = sizes.get((nT, nh))
    if need is None:
        n = ctypes.c_size_t()
        _lib.check(_lib.ising_logz_backward_workspace(plan.handle, nT, nh, ctypes.byref(n)))
        need = sizes[(nT, nh)] = n.value
    cache = plan.__dict__.setdefault("_lb", {})
    ws = cache.get(dev)
    if ws is None or ws.numel() < need:
        ws = cache[dev] = torch.empty(max(need, 8), dtype=torch.uint8, device=dev)
    gT = torch.empty(nT, dtype=torch.float64, device=dev) if want[0] else None
    gh = torch.empty(nh, dtype=torch.float64, device=dev) if want[1] else None
    gJ = torch.empty(plan.lattice.n_bonds, dtype=torch.float64, device=dev) if want[2] else None
    _lib.check(_lib.ising_logz_backward(plan.handle, g.data_ptr(), Tt.data_ptr(), nT, ht.data_ptr(), nh,
                                        lz.data_ptr(), G.data_ptr(), gT.data_ptr() if gT is not None else None,
                                        gh.data_ptr() if gh is not None else None,
                                        gJ.data_ptr() if gJ is not None else None, int(symmetric), ws.data_ptr(),
                                        ws.numel(), _stream_handle(stream)))
    return gT, gh, gJ


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------

def _lattice_struct(lat: Lattice, keep: list):
    bi = np.ascontiguousarray(lat.bond_i, dtype=np.int32)
    bj = np.ascontiguousarray(lat.bond_j, dtype=np.int32)
    bJ = np.ascontiguousarray(lat.bond_J, dtype=np.int32)
    keep += [bi, bj, bJ]
    p = _lib.i32p
    return _lib.ising_lattice(int(lat.n_spins), int(bi.shape[0]), bi.ctypes.data_as(p), bj.ctypes.data_as(p),
                              bJ.ctypes.data_as(p))


class BatchPlan:
    """Many lattices in one persistent launch (ising_batch_plan_create)."""

    def __init__(self, lattices, tune: Tune | None = None):
        self.lattices = list(lattices)
        n = len(self.lattices)
        keep: list = []
        arr = (_lib.ising_lattice * n)(*[_lattice_struct(l, keep) for l in self.lattices])
        handle = ctypes.c_void_p()
        tn = tune._c() if tune is not None else None
        _lib.check(_lib.ising_batch_plan_create(arr, n, ctypes.byref(tn) if tn is not None else None,
                                                ctypes.byref(handle)))
        self._h = handle
        off = (ctypes.c_int64 * (n + 1))()
        n_e, n_m, e_min, n_sp = ((ctypes.c_int32 * n)() for _ in range(4))
        _lib.check(_lib.ising_batch_layout(self._h, off, n_e, n_m, e_min, n_sp))
        self.offsets = np.array(off[:], dtype=np.int64)
        self.n_e = np.array(n_e[:]); self.n_m = np.array(n_m[:]); self.e_min = np.array(e_min[:])
        self.n_spins = np.array(n_sp[:])

    def __len__(self):
        return len(self.lattices)

    @property
    def handle(self):
        return self._h

    @property
    def total_configs(self) -> int:
        return int(sum(1 << int(n) for n in self.n_spins))

    def new_tables(self, device="cuda") -> torch.Tensor:
        return torch.empty(int(self.offsets[-1]), dtype=torch.uint64, device=device)

    def table(self, g_all: torch.Tensor, i: int) -> torch.Tensor:
        """Member i's [n_e][n_m] view of the concatenated tables."""
        a, b = int(self.offsets[i]), int(self.offsets[i + 1])
        return g_all[a:b].view(int(self.n_e[i]), int(self.n_m[i]))

    def close(self):
        if getattr(self, "_h", None):
            _lib.ising_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_all(plan: BatchPlan, g_all: torch.Tensor):
    if not (g_all.is_cuda and g_all.dtype == torch.uint64 and g_all.is_contiguous()
            and g_all.numel() == int(plan.offsets[-1])):
        raise ValueError(f"g_all must be a contiguous CUDA uint64 tensor of {int(plan.offsets[-1])} elements")


def batch_enumerate(plan: BatchPlan, out: torch.Tensor | None = None, stream=None,
                    symmetric: bool = False) -> torch.Tensor:
    """g(E, M) of every member, concatenated (ising_batch_enumerate); with symmetric,
    from the half of each member's configurations with its top spin up, mirrored
    M -> -M (ising_batch_enumerate_symmetric), bit-identical."""
    g = plan.new_tables() if out is None else out
    _check_all(plan, g)
    fn = _lib.ising_batch_enumerate_symmetric if symmetric else _lib.ising_batch_enumerate
    _lib.check(fn(plan.handle, g.data_ptr(), _stream_handle(stream)))
    return g


def _batch_outputs(plan: BatchPlan, Tt, ht, device):
    shape = (len(plan), Tt.numel(), ht.numel())
    return {k: torch.empty(shape, dtype=torch.float64, device=device)
            for k in ("log_z", "mean_E", "mean_M", "heat_capacity", "susceptibility")}


def batch_moments(plan: BatchPlan, g_all: torch.Tensor, T, h, stream=None) -> dict:
    """log Z and moments of every member, each [n][len(T)][len(h)] (ising_batch_moments)."""
    _check_all(plan, g_all)
    Tt, ht = _grid(T, g_all.device), _grid(h, g_all.device)
    outs = _batch_outputs(plan, Tt, ht, g_all.device)
    _lib.check(_lib.ising_batch_moments(plan.handle, g_all.data_ptr(), Tt.data_ptr(), Tt.numel(), ht.data_ptr(),
                                        ht.numel(), outs["log_z"].data_ptr(), outs["mean_E"].data_ptr(),
                                        outs["mean_M"].data_ptr(), outs["heat_capacity"].data_ptr(),
                                        outs["susceptibility"].data_ptr(), _stream_handle(stream)))
    return outs


class BatchGraph:
    """A HIP graph of {zero, batched enumeration, batched moments} with its
    buffers (ising_batch_graph_create); replay() launches it.  With symmetric
    the enumeration is the halved one (ising_batch_graph_create_symmetric)."""

    def __init__(self, plan: BatchPlan, T, h, device="cuda", symmetric: bool = False):
        self.plan = plan
        self.g_all = plan.new_tables(device)
        self.T, self.h = _grid(T, device), _grid(h, device)
        self.outs = _batch_outputs(plan, self.T, self.h, device)
        handle = ctypes.c_void_p()
        o = self.outs
        fn = _lib.ising_batch_graph_create_symmetric if symmetric else _lib.ising_batch_graph_create
        _lib.check(fn(plan.handle, self.g_all.data_ptr(), self.T.data_ptr(), self.T.numel(), self.h.data_ptr(),
                      self.h.numel(), o["log_z"].data_ptr(), o["mean_E"].data_ptr(), o["mean_M"].data_ptr(),
                      o["heat_capacity"].data_ptr(), o["susceptibility"].data_ptr(), ctypes.byref(handle)))
        self._h = handle

    def replay(self, stream=None):
        _lib.check(_lib.ising_graph_launch(self._h, _stream_handle(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.ising_graph_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
