"""Exact Ising degeneracy tables g(E, M) and partition functions on MI355X.

Enumerates all 2^N spin configurations of a finite Ising system on the GPU
(hand-written gfx950 HIP kernels behind the C-ABI library libising.so), counts
the integer degeneracy table g(E, M), and evaluates log Z(T, h) and its
moments in FP64 (Peretyatko et al., Sections 2-3, Eqs. (1)-(2)).

Importing the package does not load the GPU library; `api` (and everything
that launches work) loads it on first use and fails loudly if it is missing.
"""
from . import lattice  # noqa: F401  (inputs only; no GPU code)

__all__ = ["lattice", "api"]


def __getattr__(name):
    if name == "api":
        import importlib
        return importlib.import_module(__name__ + ".api")
    raise AttributeError(name)
