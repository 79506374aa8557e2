"""Derivatives of log Z in T, h and the couplings, in FP64, from exact counts.

Test infrastructure only (see the package docstring).

Eq. (1) gives H = E - h M with E = -sum_b J_b s_i s_j (each bond once), and
Eq. (2) gives Z = sum over configurations of exp(-H/T).  Differentiating the
definition:
  d log Z / dT     = <H> / T^2
  d log Z / dh     = <M> / T
  d log Z / dJ_b   = <s_i s_j>_b / T
  d2 log Z / dT2   = Var(H) / T^4 - 2 <H> / T^3
  d2 log Z / dT dh = (Cov(H, M) / T - <M>) / T^2
  d2 log Z / dh2   = Var(M) / T^2
with averages under the Boltzmann weights.  The T and h statistics come from
g(E, M); the bond statistics from gp (native.bond_split): gp[b](E, M) counts
the configurations of bin (E, M) whose bond-b spins agree, so the bin's sum of
s_i s_j is 2 gp - g.

A loss L = sum_{a,c} G[a, c] log Z(T_a, h_c) has dL/dJ_b = sum over
configurations of w(E, M) s_i s_j, where each configuration of bin (E, M)
carries the weight
  w(E, M) = sum_{a,c} G[a, c] exp(-(E - h_c M)/T_a - log Z(T_a, h_c)) / T_a
(its Boltzmann probability at (T_a, h_c), times G / T_a).  bin_weights gives
w; bond_grad_from_weights sums w (2 gp - g) over the bins.

Tables are dense [E - e_min][n_up], M = 2 n_up - N, as elsewhere in the oracle.
"""
from __future__ import annotations

import numpy as np

from . import thermo


def _bins(g, e_min, n_spins):
    g = np.asarray(g)
    e_idx, n_up = np.nonzero(g)
    E = (e_idx + e_min).astype(np.float64)
    M = (2 * n_up - n_spins).astype(np.float64)
    return e_idx, n_up, E, M, g[e_idx, n_up].astype(np.float64)


def log_z_derivatives(g, e_min: int, n_spins: int, T, h) -> dict:
    """First and second derivatives of log Z in (T, h), each [len(T)][len(h)]."""
    _, _, E, M, cnt = _bins(g, e_min, n_spins)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    shape = (T.shape[0], h.shape[0])
    out = {k: np.empty(shape) for k in ("d_T", "d_h", "d_TT", "d_Th", "d_hh")}
    lng = np.log(cnt)
    for a, t in enumerate(T):
        for c, hh in enumerate(h):
            H = E - hh * M
            x = lng - H / t
            w = np.exp(x - x.max())
            w /= w.sum()
            mH = (w * H).sum()
            mM = (w * M).sum()
            vH = (w * (H - mH) ** 2).sum()
            vM = (w * (M - mM) ** 2).sum()
            cHM = (w * (H - mH) * (M - mM)).sum()
            out["d_T"][a, c] = mH / t ** 2
            out["d_h"][a, c] = mM / t
            out["d_TT"][a, c] = vH / t ** 4 - 2 * mH / t ** 3
            out["d_Th"][a, c] = (cHM / t - mM) / t ** 2
            out["d_hh"][a, c] = vM / t ** 2
    return out


def bond_correlations(g, gp, e_min: int, n_spins: int, T, h) -> np.ndarray:
    """<s_i s_j> of every bond: [n_bonds][len(T)][len(h)]."""
    e_idx, n_up, E, M, cnt = _bins(g, e_min, n_spins)
    gp = np.asarray(gp)
    sig = 2.0 * gp[:, e_idx, n_up].astype(np.float64) - cnt[None, :]   # [nb][bins]
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    out = np.empty((gp.shape[0], T.shape[0], h.shape[0]))
    lng = np.log(cnt)
    for a, t in enumerate(T):
        for c, hh in enumerate(h):
            x = -(E - hh * M) / t
            x = x - (lng + x).max()
            w = np.exp(x)                     # per configuration, up to a common factor
            Z = (w * cnt).sum()
            out[:, a, c] = (sig * w[None, :]).sum(axis=1) / Z
    return out


def bond_grad(g, gp, e_min: int, n_spins: int, T, h) -> np.ndarray:
    """d log Z / dJ_b = <s_i s_j>_b / T: [n_bonds][len(T)][len(h)]."""
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    return bond_correlations(g, gp, e_min, n_spins, T, h) / T[None, :, None]


def log_z_shifted(g, gp_b, e_min: int, n_spins: int, T: float, h: float, delta: float) -> float:
    """log Z after J_b -> J_b + delta (non-integer), from the bond-b split.

    Each configuration's energy moves by -delta s_i s_j, so the sum runs over
    (E, M, s_i s_j = +-1) with counts gp and g - gp."""
    g = np.asarray(g)
    gp_b = np.asarray(gp_b)
    terms = []
    for cnt, sigma in ((gp_b, 1.0), (g - gp_b, -1.0)):
        e_idx, n_up = np.nonzero(cnt)
        E = (e_idx + e_min).astype(np.float64) - delta * sigma
        M = (2 * n_up - n_spins).astype(np.float64)
        terms.append(np.log(cnt[e_idx, n_up].astype(np.float64)) - (E - h * M) / T)
    x = np.concatenate(terms)
    mx = x.max()
    return float(mx + np.log(np.exp(x - mx).sum()))


def bin_weights(g, e_min: int, n_spins: int, T, h, G) -> np.ndarray:
    """Per-configuration weight w(E, M) of the loss sum G * log Z (see the module
    docstring); zero on empty bins.  Dense [E - e_min][n_up]."""
    g = np.asarray(g)
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    h = np.atleast_1d(np.asarray(h, dtype=np.float64))
    G = np.asarray(G, dtype=np.float64).reshape(T.shape[0], h.shape[0])
    lz = thermo.log_z(g, e_min, n_spins, T, h)
    e_idx, n_up, E, M, _ = _bins(g, e_min, n_spins)
    w = np.zeros(e_idx.shape[0])
    for a, t in enumerate(T):
        for c, hh in enumerate(h):
            w += G[a, c] * np.exp(-(E - hh * M) / t - lz[a, c]) / t
    out = np.zeros(g.shape, dtype=np.float64)
    out[e_idx, n_up] = w
    return out


def bond_grad_from_weights(g, gp, W) -> np.ndarray:
    """sum over configurations of W(bin) s_i s_j, per bond: sum_bins W (2 gp - g)."""
    g = np.asarray(g).astype(np.float64)
    gp = np.asarray(gp).astype(np.float64)
    W = np.asarray(W, dtype=np.float64)
    return ((2.0 * gp - g[None]) * W[None]).sum(axis=(1, 2))
