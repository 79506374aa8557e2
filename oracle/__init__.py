"""CPU oracle for the exact Ising degeneracy table and partition function.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything here.  The library never
does; it shares no code, header, table or helper with this package.

Contents (each function cites the passage of Peretyatko et al. it follows):
  native.count_range / count_all  the definition of g(E, M) (Section 2, Eq. (1)
                                  and the multiplicity statement after Eq. (2)),
                                  brute force over configurations, in C;
  native.tm_torus                 exact row transfer-matrix count for square tori
                                  with per-bond couplings (independent algorithm);
  bruteforce.g_numpy              the same definition vectorised in numpy (small N);
  native.bond_split               g plus, per bond, the count of configurations
                                  of each (E, M) whose two spins agree, brute force
                                  in C (derivatives in the couplings of Eq. (1));
  thermo.log_z / moments          Eq. (2) evaluated from g in FP64;
  grad                            first and second derivatives of log Z in T and
                                  h, per-bond d log Z / dJ_b, log Z at a shifted
                                  non-integer coupling, and the per-configuration
                                  weights of a loss sum G * log Z, in FP64;
  closed_forms                    1D ring and Kaufman torus closed forms (pins).

Every function here is pinned by a test against something other than itself:
the paper's Table 1, closed forms, invariants, brute force on tiny inputs.
"""
from . import closed_forms, native, thermo, bruteforce, grad  # noqa: F401

__all__ = ["closed_forms", "native", "thermo", "bruteforce", "grad"]
