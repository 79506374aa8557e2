"""ctypes binding of libising.so: the C ABI of include/ising.h, same names.

Argument marshalling only; all work runs in the library's HIP kernels.
Importing this module fails loudly if libising.so has not been built.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# ISING_LIBRARY may name another build of the same library (e.g. a debug build).
LIB_PATH = os.environ.get("ISING_LIBRARY") or os.path.join(_HERE, "libising.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1110_2561_amd.build` "
                      "(there is no CPU fallback)")

lib = ctypes.CDLL(LIB_PATH)

i32 = ctypes.c_int32
u64 = ctypes.c_uint64
i32p = ctypes.POINTER(ctypes.c_int32)
u64p = ctypes.POINTER(ctypes.c_uint64)
vp = ctypes.c_void_p

ISING_OK = 0
STATUS = {0: "ISING_OK", -1: "ISING_EINVAL", -2: "ISING_ETOO_MANY_SPINS", -3: "ISING_EBOND",
          -4: "ISING_ERANGE", -5: "ISING_EHIP", -6: "ISING_ENOMEM", -7: "ISING_EUNSUPPORTED"}


class ising_lattice(ctypes.Structure):
    _fields_ = [("n_spins", i32), ("n_bonds", i32), ("bond_i", i32p), ("bond_j", i32p), ("bond_J", i32p)]


class ising_tune(ctypes.Structure):
    _fields_ = [("inner_bits", i32), ("tile_bits", i32), ("waves_per_block", i32), ("replicas", i32),
                ("max_blocks", i32), ("prefix_bits", i32)]


class IsingError(RuntimeError):
    def __init__(self, code: int, detail: str):
        name = STATUS.get(code, str(code))
        super().__init__(detail if detail.startswith(name) else f"{name}: {detail}")
        self.code = code


def _sig(name, restype, *args):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = list(args)
    return f


ising_plan_create = _sig("ising_plan_create", i32, ctypes.POINTER(ising_lattice), ctypes.POINTER(ising_tune),
                         ctypes.POINTER(vp))
ising_plan_destroy = _sig("ising_plan_destroy", i32, vp)
ising_hist_shape = _sig("ising_hist_shape", i32, vp, i32p, i32p, i32p)
ising_plan_layout = _sig("ising_plan_layout", i32, vp, i32p, i32p, i32p, u64p)
ising_enumerate = _sig("ising_enumerate", i32, vp, vp, vp)
ising_enumerate_range = _sig("ising_enumerate_range", i32, vp, u64, u64, vp, vp)
ising_enumerate_symmetric = _sig("ising_enumerate_symmetric", i32, vp, vp, vp)
ising_logz = _sig("ising_logz", i32, vp, i32, i32, i32, i32, vp, i32, vp, i32, vp, vp)
ising_moments = _sig("ising_moments", i32, vp, i32, i32, i32, i32, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp)
ising_logz_derivatives = _sig("ising_logz_derivatives", i32, vp, i32, i32, i32, i32, vp, i32, vp, i32, vp, vp, vp,
                              vp, vp, vp, vp)
ising_bin_weights = _sig("ising_bin_weights", i32, vp, i32, i32, i32, i32, vp, i32, vp, i32, vp, vp, vp, vp)
ising_bond_workspace = _sig("ising_bond_workspace", i32, vp, ctypes.POINTER(ctypes.c_size_t))
ising_bond_backward = _sig("ising_bond_backward", i32, vp, vp, vp, vp, ctypes.c_size_t, vp)
ising_bond_backward_symmetric = _sig("ising_bond_backward_symmetric", i32, vp, vp, vp, vp, ctypes.c_size_t, vp)
ising_bond_backward_noalloc = _sig("ising_bond_backward_noalloc", i32, vp, vp, vp, vp)
ising_logz_backward_workspace = _sig("ising_logz_backward_workspace", i32, vp, i32, i32,
                                     ctypes.POINTER(ctypes.c_size_t))
ising_logz_backward = _sig("ising_logz_backward", i32, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp, i32, vp,
                           ctypes.c_size_t, vp)
i64p = ctypes.POINTER(ctypes.c_int64)
ising_batch_plan_create = _sig("ising_batch_plan_create", i32, ctypes.POINTER(ising_lattice), i32,
                               ctypes.POINTER(ising_tune), ctypes.POINTER(vp))
ising_batch_plan_destroy = _sig("ising_batch_plan_destroy", i32, vp)
ising_batch_layout = _sig("ising_batch_layout", i32, vp, i64p, i32p, i32p, i32p, i32p)
ising_batch_enumerate = _sig("ising_batch_enumerate", i32, vp, vp, vp)
ising_batch_enumerate_symmetric = _sig("ising_batch_enumerate_symmetric", i32, vp, vp, vp)
ising_batch_moments = _sig("ising_batch_moments", i32, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp, vp)
ising_batch_graph_create = _sig("ising_batch_graph_create", i32, vp, vp, vp, i32, vp, i32, vp, vp, vp, vp, vp,
                                ctypes.POINTER(vp))
ising_batch_graph_create_symmetric = _sig("ising_batch_graph_create_symmetric", i32, vp, vp, vp, i32, vp, i32, vp,
                                          vp, vp, vp, vp, ctypes.POINTER(vp))
ising_graph_launch = _sig("ising_graph_launch", i32, vp, vp)
ising_graph_destroy = _sig("ising_graph_destroy", i32, vp)
ising_status_str = _sig("ising_status_str", ctypes.c_char_p, i32)
ising_last_error = _sig("ising_last_error", ctypes.c_char_p)
ising_version = _sig("ising_version", ctypes.c_char_p)


def check(code: int) -> None:
    """Raise IsingError for a nonzero status, with the library's message."""
    if code != ISING_OK:
        raise IsingError(code, ising_last_error().decode())
