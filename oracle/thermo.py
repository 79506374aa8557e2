"""FP64 evaluation of Eq. (2) and its moments from a degeneracy table.

Test infrastructure only (see the package docstring).

Eq. (2) sums exp(-H/T) over all configurations; grouping configurations by
(E, M) turns it into Z(T, h) = sum_{E,M} g(E, M) exp(-(E - h M)/T), with
H = E - h M from Eq. (1) (k_B = 1).  log Z is evaluated as a log-sum-exp over
the nonzero bins: a = ln g - (E - h M)/T, log Z = max(a) + ln sum exp(a - max(a)).

Moments, under the Boltzmann weights p = g exp(-(E - hM)/T) / Z:
  <E>  mean exchange energy,  <M>  mean spin excess,
  C    = Var(E - h M) / T^2   (heat capacity at fixed h, total not per spin),
  chi  = Var(M) / T           (susceptibility, total not per spin),
with variances from centred second passes.

Dense table layout: g[E - e_min][n_up], M = 2 n_up - N.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def _bins(g: np.ndarray, e_min: int, n_spins: int):
    g = np.asarray(g)
    e_idx, n_up = np.nonzero(g)
    E = (e_idx + e_min).astype(np.float64)
    M = (2 * n_up - n_spins).astype(np.float64)
    lng = np.log(g[e_idx, n_up].astype(np.float64))
    return E, M, lng


def log_z(g: np.ndarray, e_min: int, n_spins: int, T, h) -> np.ndarray:
    """log Z [len(T)][len(h)] in FP64."""
    E, M, lng = _bins(g, e_min, n_spins)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    out = np.empty((T.shape[0], h.shape[0]))
    for a, t in enumerate(T):
        for b, hh in enumerate(h):
            x = lng - (E - hh * M) / t
            mx = x.max()
            out[a, b] = mx + np.log(np.exp(x - mx).sum())
    return out


def moments(g: np.ndarray, e_min: int, n_spins: int, T, h):
    """(<E>, <M>, C, chi), each [len(T)][len(h)] in FP64."""
    E, M, lng = _bins(g, e_min, n_spins)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    shape = (T.shape[0], h.shape[0])
    mE, mM, C, chi = (np.empty(shape) for _ in range(4))
    for a, t in enumerate(T):
        for b, hh in enumerate(h):
            x = lng - (E - hh * M) / t
            w = np.exp(x - x.max())
            Z = w.sum()
            e1 = (w * E).sum() / Z
            m1 = (w * M).sum() / Z
            H = E - hh * M
            h1 = e1 - hh * m1
            mE[a, b] = e1
            mM[a, b] = m1
            C[a, b] = (w * (H - h1) ** 2).sum() / Z / (t * t)
            chi[a, b] = (w * (M - m1) ** 2).sum() / Z / t
    return mE, mM, C, chi


def log_z_mp(g: np.ndarray, e_min: int, n_spins: int, T: float, h: float, dps: int = 50):
    """log Z of one (T, h) with mpmath at `dps` digits (rounding reference)."""
    g = np.asarray(g)
    e_idx, n_up = np.nonzero(g)
    with mp.workdps(dps):
        T = mp.mpf(T); h = mp.mpf(h)
        Z = mp.mpf(0)
        for e, n in zip(e_idx.tolist(), n_up.tolist()):
            E = e + e_min
            M = 2 * n - n_spins
            Z += mp.mpf(int(g[e, n])) * mp.exp(-(E - h * M) / T)
        return mp.log(Z)
