"""Closed forms that pin the oracle from outside (test infrastructure only).

These are textbook results, not part of the paper's method; they are used to
check the oracle's counts and its FP64 evaluation of Eq. (2).

* 1D ring (Ising's 1925 solution, cited in the paper's introduction):
  - degeneracies: a cyclic sequence of N spins with n_up up-spins split into r
    runs of ups (and r runs of downs) has 2r unsatisfied bonds, so
    E = -N + 4r.  The number of such sequences is
    (N / r) * C(n_up - 1, r - 1) * C(N - n_up - 1, r - 1);
  - Z(T, h) = lam_+^N + lam_-^N with
    lam_pm = e^K cosh(h/T) pm sqrt(e^{2K} sinh^2(h/T) + e^{-2K}), K = J/T.
* Square m x n torus at h = 0 (Kaufman 1949, the finite-lattice form of
  Onsager's solution):
  Z = 1/2 (2 sinh 2K)^{mn/2} (Z1 + Z2 + Z3 + Z4),
  Z1 = prod_{r<n} 2 cosh(m g_{2r+1}/2),  Z2 = prod_{r<n} 2 sinh(m g_{2r+1}/2),
  Z3 = prod_{r<n} 2 cosh(m g_{2r}/2),    Z4 = prod_{r<n} 2 sinh(m g_{2r}/2),
  cosh g_l = cosh 2K coth 2K - cos(l pi / n) for l >= 1 (g_l > 0), and the
  signed g_0 = 2K + ln tanh K.  m counts rows and n the sites per row.

Evaluated with mpmath at 50 significant digits or more.
"""
from __future__ import annotations

from math import comb

import mpmath as mp
import numpy as np

_DPS = 50


def _prec():
    # Never below 50 digits, and never below what a caller (for instance
    # mpmath's numerical differentiation) has already raised the precision to.
    return mp.workprec(max(mp.mp.prec, int(_DPS * 3.33) + 8))


def ring_g(N: int) -> np.ndarray:
    """Dense g [2N+1][N+1] of the uniform J = 1 ring (row E + N, column n_up)."""
    if N < 3:
        raise ValueError("ring needs N >= 3")
    g = np.zeros((2 * N + 1, N + 1), dtype=np.uint64)
    g[0, 0] = 1  # all down: E = -N
    g[0, N] = 1  # all up
    for n_up in range(1, N):
        for r in range(1, min(n_up, N - n_up) + 1):
            num = N * comb(n_up - 1, r - 1) * comb(N - n_up - 1, r - 1)
            assert num % r == 0
            g[(-N + 4 * r) + N, n_up] += num // r
    return g


def ring_logz(N: int, T: float, h: float, J: float = 1.0) -> mp.mpf:
    with _prec():
        T = mp.mpf(T); h = mp.mpf(h); K = mp.mpf(J) / T; x = h / T
        root = mp.sqrt(mp.exp(2 * K) * mp.sinh(x) ** 2 + mp.exp(-2 * K))
        lp = mp.exp(K) * mp.cosh(x) + root
        lm = mp.exp(K) * mp.cosh(x) - root
        return mp.log(lp ** N + lm ** N)


def kaufman_logz(m: int, n: int, T: float) -> mp.mpf:
    """log Z of the m x n square torus, J = 1, h = 0."""
    with _prec():
        K = 1 / mp.mpf(T)
        c = mp.cosh(2 * K) * mp.coth(2 * K)

        def gam(l):
            if l == 0:
                return 2 * K + mp.log(mp.tanh(K))
            return mp.acosh(c - mp.cos(l * mp.pi / n))

        z1 = z2 = z3 = z4 = mp.mpf(1)
        for r in range(n):
            go = gam(2 * r + 1)
            ge = gam(2 * r)
            z1 *= 2 * mp.cosh(m * go / 2)
            z2 *= 2 * mp.sinh(m * go / 2)
            z3 *= 2 * mp.cosh(m * ge / 2)
            z4 *= 2 * mp.sinh(m * ge / 2)
        Z = (2 * mp.sinh(2 * K)) ** (mp.mpf(m * n) / 2) * (z1 + z2 + z3 + z4) / 2
        return mp.log(Z)


def binomial_marginal(N: int) -> np.ndarray:
    """sum_E g(E, M) = C(N, n_up), the statement closing Section 2."""
    return np.array([comb(N, k) for k in range(N + 1)], dtype=object)
