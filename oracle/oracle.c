/*
 * CPU oracle for the exact Ising degeneracy table g(E, M).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library calls, links or loads
 * this file; it exists so that the tests and the benchmark's CPU baseline can
 * check the GPU path against an independent, obviously correct computation.
 * It shares no code, header or table with the GPU path.
 *
 * Definitions followed (Peretyatko et al., Section 2):
 *   - Eq. (1): H = -(1/2) sum_i sum_{j in nbr(i)} J_ij S_i S_j - h sum_i S_i.
 *     The 1/2 over the double neighbour sum counts every bond once, so for a
 *     bond multiset the exchange energy is E = -sum_b J_b s_i s_j.
 *   - Every one of the 2^N configurations is assigned the pair (E, M), where
 *     M is the spin excess sum_i s_i; g(E, M) is the number of configurations
 *     with that pair (the degeneracy multiplicity discussed after Eq. (2)).
 *   - Section 3a: the spin excess follows from the number of "up" bits.
 *
 * Conventions: configuration index c in [0, 2^N); bit u of c set means
 * s_u = +1.  n_up = popcount(c), M = 2 n_up - N.  Output table g is dense,
 * row-major [2S+1][N+1], row E + S, column n_up, S = sum_b |J_b|.
 *
 * Three exact counts live here:
 *   oracle_count_range : the definition written out (loop over configurations,
 *                        loop over bonds), for an index range of configurations;
 *   oracle_tm_torus    : a row-to-row transfer-matrix count for square tori with
 *                        per-bond couplings (a different algorithm, used to pin
 *                        the brute force and to reach the 6x6 / 8x5 sizes);
 *   oracle_bond_split  : g together with, for every bond, the count of the
 *                        configurations of each (E, n_up) whose two spins agree
 *                        (the statistics behind derivatives in the couplings);
 *   oracle_band_count  : a count along the site order for lattices whose bonds
 *                        join sites at most B apart (a third algorithm, for
 *                        free-boundary patches too large to enumerate);
 *   oracle_row_words   : the paper's own scheme (Section 3) for the square
 *                        torus with couplings +-1: the lattice as one bit
 *                        word per row, satisfied bonds counted with XOR, NOT,
 *                        a mask and popcount (and, for J = -1 bonds, one more
 *                        XOR with the row's sign mask), E = 2 (N - En), M from
 *                        popcounts.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

/* ---------------------------------------------------------------------- */
/* Brute force: the definition, configuration by configuration.           */
/* ---------------------------------------------------------------------- */

typedef struct {
  int n, nb;
  const int32_t *bi, *bj, *bJ;
  int64_t S;
  uint64_t lo, hi;
  uint64_t *table; /* private [2S+1][n+1] */
} count_job;

static void *count_worker(void *arg) {
  count_job *jb = (count_job *)arg;
  const int nm = jb->n + 1;
  for (uint64_t c = jb->lo; c < jb->hi; ++c) {
    int64_t e = 0;
    for (int b = 0; b < jb->nb; ++b) {
      const int64_t si = ((c >> jb->bi[b]) & 1u) ? 1 : -1;
      const int64_t sj = ((c >> jb->bj[b]) & 1u) ? 1 : -1;
      e -= (int64_t)jb->bJ[b] * si * sj;
    }
    int up = 0;
    for (int u = 0; u < jb->n; ++u) up += (int)((c >> u) & 1u);
    jb->table[(size_t)(e + jb->S) * nm + up] += 1;
  }
  return NULL;
}

/* Count configurations with index in [first, first + count) into g (added,
 * not overwritten).  Returns 0 on success, <0 on bad arguments.  For n = 64
 * the range must end before the last configuration (indices are uint64). */
int oracle_count_range(int n, int nb, const int32_t *bi, const int32_t *bj,
                       const int32_t *bJ, uint64_t first, uint64_t count,
                       int n_threads, uint64_t *g) {
  if (n < 1 || n > 64 || nb < 0 || n_threads < 1 || !g) return -1;
  int64_t S = 0;
  for (int b = 0; b < nb; ++b) {
    if (bi[b] < 0 || bi[b] >= n || bj[b] < 0 || bj[b] >= n) return -2;
    S += bJ[b] < 0 ? -(int64_t)bJ[b] : bJ[b];
  }
  if (n < 64) {
    const uint64_t total = (uint64_t)1 << n;
    if (first > total || count > total - first) return -3;
  } else if (count > UINT64_MAX - first) {
    return -3;
  }
  const size_t cells = (size_t)(2 * S + 1) * (size_t)(n + 1);
  if (count == 0) return 0;
  if ((uint64_t)n_threads > count) n_threads = (int)count;

  count_job *jobs = (count_job *)calloc((size_t)n_threads, sizeof(count_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -4; }
  const uint64_t per = count / (uint64_t)n_threads, rem = count % (uint64_t)n_threads;
  uint64_t lo = first;
  int rc = 0;
  for (int t = 0; t < n_threads; ++t) {
    const uint64_t len = per + ((uint64_t)t < rem ? 1 : 0);
    jobs[t] = (count_job){n, nb, bi, bj, bJ, S, lo, lo + len,
                          (uint64_t *)calloc(cells, sizeof(uint64_t))};
    if (!jobs[t].table) { rc = -4; n_threads = t; break; }
    lo += len;
  }
  if (rc == 0) {
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, count_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    for (int t = 0; t < n_threads; ++t)
      for (size_t k = 0; k < cells; ++k) g[k] += jobs[t].table[k];
  }
  for (int t = 0; t < n_threads; ++t) free(jobs[t].table);
  free(jobs); free(th);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Transfer matrix for an Lx x Ly square torus with per-bond couplings.     */
/* ---------------------------------------------------------------------- */
/* Site (x, y) is index y*Lx + x.  Jh[y*Lx + x] couples (x, y)-(x+1 mod Lx, y);
 * Jv[y*Lx + x] couples (x, y)-(x, y+1 mod Ly).  A row state r has bit x set
 * when s(x, y) = +1.  Fixing the first row a, F[r] is the (E, n_up) count of
 * rows 0..y with row y in state r; adding a row adds its in-row bonds and the
 * vertical bonds to the previous row; the last row closes onto row a. */

static int64_t row_energy(int Lx, const int32_t *Jh_row, unsigned r) {
  int64_t e = 0;
  for (int x = 0; x < Lx; ++x) {
    const int64_t s1 = ((r >> x) & 1u) ? 1 : -1;
    const int64_t s2 = ((r >> ((x + 1) % Lx)) & 1u) ? 1 : -1;
    e -= (int64_t)Jh_row[x] * s1 * s2;
  }
  return e;
}

static int64_t link_energy(int Lx, const int32_t *Jv_row, unsigned r_lo, unsigned r_hi) {
  int64_t e = 0;
  for (int x = 0; x < Lx; ++x) {
    const int64_t s1 = ((r_lo >> x) & 1u) ? 1 : -1;
    const int64_t s2 = ((r_hi >> x) & 1u) ? 1 : -1;
    e -= (int64_t)Jv_row[x] * s1 * s2;
  }
  return e;
}

typedef struct {
  int Lx, Ly;
  const int32_t *Jh, *Jv;
  int64_t S;
  unsigned a_lo, a_hi;     /* first-row states handled by this worker */
  uint64_t *table;         /* private [2S+1][N+1] */
  int status;
} tm_job;

static void *tm_worker(void *arg) {
  tm_job *jb = (tm_job *)arg;
  const int Lx = jb->Lx, Ly = jb->Ly, N = Lx * Ly, nm = N + 1;
  const unsigned R = 1u << Lx;
  const int64_t ne = 2 * jb->S + 1;
  const size_t poly = (size_t)ne * (size_t)nm;
  uint64_t *F = (uint64_t *)malloc(sizeof(uint64_t) * poly * R);
  uint64_t *G = (uint64_t *)malloc(sizeof(uint64_t) * poly * R);
  int64_t *eintra = (int64_t *)malloc(sizeof(int64_t) * R * (size_t)Ly);
  if (!F || !G || !eintra) { free(F); free(G); free(eintra); jb->status = -4; return NULL; }
  for (int y = 0; y < Ly; ++y)
    for (unsigned r = 0; r < R; ++r) eintra[(size_t)y * R + r] = row_energy(Lx, jb->Jh + y * Lx, r);

  for (unsigned a = jb->a_lo; a < jb->a_hi; ++a) {
    memset(F, 0, sizeof(uint64_t) * poly * R);
    F[(size_t)a * poly + (size_t)(eintra[a] + jb->S) * nm + __builtin_popcount(a)] = 1;
    for (int y = 1; y < Ly; ++y) {
      memset(G, 0, sizeof(uint64_t) * poly * R);
      for (unsigned r = 0; r < R; ++r) {
        const uint64_t *src = F + (size_t)r * poly;
        for (unsigned r2 = 0; r2 < R; ++r2) {
          const int64_t de = eintra[(size_t)y * R + r2] + link_energy(Lx, jb->Jv + (y - 1) * Lx, r, r2);
          const int dn = __builtin_popcount(r2);
          uint64_t *dst = G + (size_t)r2 * poly;
          for (int64_t e = 0; e < ne; ++e) {
            const int64_t e2 = e + de;
            if (e2 < 0 || e2 >= ne) continue;
            const uint64_t *s = src + (size_t)e * nm;
            uint64_t *d = dst + (size_t)e2 * nm;
            for (int n = 0; n + dn < nm; ++n) d[n + dn] += s[n];
          }
        }
      }
      uint64_t *t = F; F = G; G = t;
    }
    for (unsigned r = 0; r < R; ++r) {
      const int64_t de = link_energy(Lx, jb->Jv + (Ly - 1) * Lx, r, a);
      const uint64_t *src = F + (size_t)r * poly;
      for (int64_t e = 0; e < ne; ++e) {
        const int64_t e2 = e + de;
        if (e2 < 0 || e2 >= ne) continue;
        for (int n = 0; n < nm; ++n) jb->table[(size_t)e2 * nm + n] += src[(size_t)e * nm + n];
      }
    }
  }
  free(F); free(G); free(eintra);
  return NULL;
}

/* Exact g for the torus into g (overwritten), S = sum |Jh| + sum |Jv|. */
int oracle_tm_torus(int Lx, int Ly, const int32_t *Jh, const int32_t *Jv,
                    int n_threads, uint64_t *g) {
  if (Lx < 2 || Ly < 2 || Lx > 16 || Lx * Ly > 62 || n_threads < 1 || !g) return -1;
  int64_t S = 0;
  for (int k = 0; k < Lx * Ly; ++k) {
    S += Jh[k] < 0 ? -(int64_t)Jh[k] : Jh[k];
    S += Jv[k] < 0 ? -(int64_t)Jv[k] : Jv[k];
  }
  const int N = Lx * Ly;
  const size_t cells = (size_t)(2 * S + 1) * (size_t)(N + 1);
  const unsigned R = 1u << Lx;
  if ((unsigned)n_threads > R) n_threads = (int)R;
  tm_job *jobs = (tm_job *)calloc((size_t)n_threads, sizeof(tm_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -4; }
  int rc = 0, made = 0;
  for (int t = 0; t < n_threads; ++t) {
    const unsigned lo = (unsigned)((uint64_t)R * t / n_threads);
    const unsigned hi = (unsigned)((uint64_t)R * (t + 1) / n_threads);
    jobs[t] = (tm_job){Lx, Ly, Jh, Jv, S, lo, hi, (uint64_t *)calloc(cells, sizeof(uint64_t)), 0};
    if (!jobs[t].table) { rc = -4; break; }
    made = t + 1;
  }
  if (rc == 0) {
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, tm_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    memset(g, 0, cells * sizeof(uint64_t));
    for (int t = 0; t < n_threads; ++t) {
      if (jobs[t].status) rc = jobs[t].status;
      for (size_t k = 0; k < cells; ++k) g[k] += jobs[t].table[k];
    }
  }
  for (int t = 0; t < made; ++t) free(jobs[t].table);
  free(jobs); free(th);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Bond-resolved counts.                                                    */
/* ---------------------------------------------------------------------- */
/* H of Eq. (1) depends on the coupling of bond b only through -J_b s_i s_j,
 * so derivatives in J_b need, per (E, M), how many configurations have
 * s_i s_j = +1 on that bond.  gp[b][E + S][n_up] counts them (the rest of the
 * bin, g - gp, has s_i s_j = -1).  Same loops as the brute force above. */

typedef struct {
  int n, nb;
  const int32_t *bi, *bj, *bJ;
  int64_t S;
  uint64_t lo, hi;
  uint64_t *table; /* private g   [2S+1][n+1]      */
  uint64_t *split; /* private gp  [nb][2S+1][n+1]  */
  unsigned char *agree;
} split_job;

static void *split_worker(void *arg) {
  split_job *jb = (split_job *)arg;
  const int nm = jb->n + 1;
  const size_t cells = (size_t)(2 * jb->S + 1) * (size_t)nm;
  for (uint64_t c = jb->lo; c < jb->hi; ++c) {
    int64_t e = 0;
    for (int b = 0; b < jb->nb; ++b) {
      const int64_t si = ((c >> jb->bi[b]) & 1u) ? 1 : -1;
      const int64_t sj = ((c >> jb->bj[b]) & 1u) ? 1 : -1;
      e -= (int64_t)jb->bJ[b] * si * sj;
      jb->agree[b] = (unsigned char)(si == sj);
    }
    int up = 0;
    for (int u = 0; u < jb->n; ++u) up += (int)((c >> u) & 1u);
    const size_t cell = (size_t)(e + jb->S) * nm + up;
    jb->table[cell] += 1;
    for (int b = 0; b < jb->nb; ++b)
      if (jb->agree[b]) jb->split[(size_t)b * cells + cell] += 1;
  }
  return NULL;
}

/* g (overwritten) and gp (overwritten) over all 2^n configurations. */
int oracle_bond_split(int n, int nb, const int32_t *bi, const int32_t *bj, const int32_t *bJ,
                      int n_threads, uint64_t *g, uint64_t *gp) {
  if (n < 1 || n > 40 || nb < 0 || n_threads < 1 || !g || (nb > 0 && !gp)) return -1;
  int64_t S = 0;
  for (int b = 0; b < nb; ++b) {
    if (bi[b] < 0 || bi[b] >= n || bj[b] < 0 || bj[b] >= n) return -2;
    S += bJ[b] < 0 ? -(int64_t)bJ[b] : bJ[b];
  }
  const uint64_t total = (uint64_t)1 << n;
  const size_t cells = (size_t)(2 * S + 1) * (size_t)(n + 1);
  if ((uint64_t)n_threads > total) n_threads = (int)total;
  split_job *jobs = (split_job *)calloc((size_t)n_threads, sizeof(split_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -4; }
  const uint64_t per = total / (uint64_t)n_threads, rem = total % (uint64_t)n_threads;
  uint64_t lo = 0;
  int rc = 0, made = 0;
  for (int t = 0; t < n_threads; ++t) {
    const uint64_t len = per + ((uint64_t)t < rem ? 1 : 0);
    jobs[t] = (split_job){n, nb, bi, bj, bJ, S, lo, lo + len,
                          (uint64_t *)calloc(cells, sizeof(uint64_t)),
                          (uint64_t *)calloc(cells * (size_t)(nb > 0 ? nb : 1), sizeof(uint64_t)),
                          (unsigned char *)calloc((size_t)(nb > 0 ? nb : 1), 1)};
    made = t + 1;
    if (!jobs[t].table || !jobs[t].split || !jobs[t].agree) { rc = -4; break; }
    lo += len;
  }
  if (rc == 0) {
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, split_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    memset(g, 0, cells * sizeof(uint64_t));
    if (nb > 0) memset(gp, 0, cells * (size_t)nb * sizeof(uint64_t));
    for (int t = 0; t < n_threads; ++t) {
      for (size_t k = 0; k < cells; ++k) g[k] += jobs[t].table[k];
      for (size_t k = 0; k < cells * (size_t)nb; ++k) gp[k] += jobs[t].split[k];
    }
  }
  for (int t = 0; t < made; ++t) { free(jobs[t].table); free(jobs[t].split); free(jobs[t].agree); }
  free(jobs); free(th);
  return rc;
}

/* ---------------------------------------------------------------------- */
/* Banded count: sites in index order, bonds at most B sites apart.         */
/* ---------------------------------------------------------------------- */
/* Adding site k with spin s_k adds -J s_i s_k for its bonds to earlier sites
 * i >= k - B (Eq. (1), each bond once, at its later end), and 1 to n_up if
 * s_k = +1.  So the counts of the first k + 1 spins need only the spins of the
 * last B sites: F_k[state][E + S][n_up], state bit d - 1 = spin of site k - d
 * (d = 1..B; bit set = +1).  Summing F_{N-1} over the states gives g.  Exact
 * integer arithmetic throughout.  Returns -1 on bad input, -2 if the
 * bandwidth exceeds 20, -3 if the tables would exceed 2^28 entries, -4 if
 * out of memory. */
int oracle_band_count(int n, int nb, const int32_t *bi, const int32_t *bj, const int32_t *bJ, uint64_t *g) {
  if (n < 1 || n > 64 || nb < 0 || !g) return -1;
  int64_t S = 0;
  int B = 0;
  for (int b = 0; b < nb; ++b) {
    if (bi[b] < 0 || bi[b] >= n || bj[b] < 0 || bj[b] >= n || bi[b] == bj[b]) return -1;
    S += bJ[b] < 0 ? -(int64_t)bJ[b] : bJ[b];
    const int d = bi[b] > bj[b] ? bi[b] - bj[b] : bj[b] - bi[b];
    if (d > B) B = d;
  }
  if (B > 20) return -2;
  const int64_t ne = 2 * S + 1, nm = n + 1;
  const size_t cells = (size_t)ne * (size_t)nm;
  const size_t states = (size_t)1 << B;
  if ((double)states * (double)cells > (double)((size_t)1 << 28)) return -3;
  /* bonds grouped by their later end: (distance, coupling) */
  int *cnt = (int *)calloc((size_t)n, sizeof(int));
  int *start = (int *)calloc((size_t)n + 1, sizeof(int));
  int *dist = (int *)malloc(sizeof(int) * (size_t)(nb > 0 ? nb : 1));
  int64_t *cJ = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nb > 0 ? nb : 1));
  uint64_t *F = (uint64_t *)calloc(states * cells, sizeof(uint64_t));
  uint64_t *G = (uint64_t *)calloc(states * cells, sizeof(uint64_t));
  if (!cnt || !start || !dist || !cJ || !F || !G) {
    free(cnt); free(start); free(dist); free(cJ); free(F); free(G);
    return -4;
  }
  for (int b = 0; b < nb; ++b) ++cnt[bi[b] > bj[b] ? bi[b] : bj[b]];
  for (int k = 0; k < n; ++k) start[k + 1] = start[k] + cnt[k];
  memset(cnt, 0, sizeof(int) * (size_t)n);
  for (int b = 0; b < nb; ++b) {
    const int hi = bi[b] > bj[b] ? bi[b] : bj[b], lo = bi[b] > bj[b] ? bj[b] : bi[b];
    const int slot = start[hi] + cnt[hi]++;
    dist[slot] = hi - lo;
    cJ[slot] = bJ[b];
  }
  const size_t mask = states - 1;
  F[(size_t)S * (size_t)nm] = 1;           /* no spins yet: state 0, E = 0, n_up = 0 */
  for (int k = 0; k < n; ++k) {
    memset(G, 0, sizeof(uint64_t) * states * cells);
    for (size_t st = 0; st < states; ++st) {
      const uint64_t *src = F + st * cells;
      for (int s = 0; s <= 1; ++s) {
        const int64_t sk = s ? 1 : -1;
        int64_t de = 0;
        for (int q = start[k]; q < start[k + 1]; ++q) {
          const int64_t si = ((st >> (dist[q] - 1)) & 1u) ? 1 : -1;
          de -= cJ[q] * si * sk;
        }
        const size_t ns = B ? (((st << 1) | (size_t)s) & mask) : 0;
        uint64_t *dst = G + ns * cells;
        for (int64_t e = 0; e < ne; ++e) {
          const int64_t e2 = e + de;
          if (e2 < 0 || e2 >= ne) continue;
          const uint64_t *a = src + (size_t)e * (size_t)nm;
          uint64_t *c = dst + (size_t)e2 * (size_t)nm;
          for (int u = 0; u + s < nm; ++u) c[u + s] += a[u];
        }
      }
    }
    uint64_t *t = F; F = G; G = t;
  }
  memset(g, 0, sizeof(uint64_t) * cells);
  for (size_t st = 0; st < states; ++st)
    for (size_t c = 0; c < cells; ++c) g[c] += F[st * cells + c];
  free(cnt); free(start); free(dist); free(cJ); free(F); free(G);
  return 0;
}

/* ---------------------------------------------------------------------- */
/* The paper's scheme for the square torus with couplings +-1 (Section 3a-c). */
/* ---------------------------------------------------------------------- */
/* A configuration is Ly words of Lx bits, word r = row r (site (x, r) is bit
 * x, index r * Lx + x, so the word values are the configuration index split
 * into Lx-bit pieces).  A bond is satisfied when J s_i s_j = +1: for J = 1
 * when its spins agree, for J = -1 when they differ (Eq. (1) allows
 * sign-changing couplings, Section 2).  Satisfied bonds En: within a row,
 * XOR of the word with itself rotated by one bit, NOT, then XOR with the
 * row's mask of J = -1 bonds, keep the Lx significant bits, popcount
 * (Section 3b's row pass, on the row's periodic ring); between rows r and
 * r + 1 (mod Ly) the same with the two words and the vertical sign mask
 * (Section 3c).  With 2N bonds of |J| = 1, E = (2N - En) - En = 2 (N - En)
 * (Section 3c), and the up count is the sum of the words' popcounts
 * (Section 3a).  With all couplings 1 the sign masks are zero and this is
 * the paper's J = 1 scheme unchanged. */

typedef struct {
  int Lx, Ly;
  uint64_t lo, hi;
  const uint64_t *neg_h, *neg_v;   /* per row: bit x set when that bond has J = -1 */
  uint64_t *table;   /* private [4N + 1][N + 1] */
} words_job;

static void *words_worker(void *arg) {
  words_job *jb = (words_job *)arg;
  const int Lx = jb->Lx, Ly = jb->Ly, N = Lx * Ly, nm = N + 1;
  const uint64_t mask = (Lx == 64) ? ~0ull : ((1ull << Lx) - 1);
  uint64_t a[64];
  for (uint64_t c = jb->lo; c < jb->hi; ++c) {
    int En = 0, up = 0;
    for (int r = 0; r < Ly; ++r) a[r] = (c >> (r * Lx)) & mask;
    for (int r = 0; r < Ly; ++r) {
      const uint64_t rot = ((a[r] >> 1) | (a[r] << (Lx - 1))) & mask;     /* bit x <- bit x + 1 (mod Lx) */
      En += __builtin_popcountll((~(a[r] ^ rot) ^ jb->neg_h[r]) & mask);
      En += __builtin_popcountll((~(a[r] ^ a[(r + 1) % Ly]) ^ jb->neg_v[r]) & mask);
      up += __builtin_popcountll(a[r]);
    }
    const int E = 2 * (N - En);
    jb->table[(size_t)(E + 2 * N) * (size_t)nm + (size_t)up] += 1;
  }
  return NULL;
}

/* Counts of configurations [first, first + count) of the Lx x Ly torus with
 * couplings +-1, into g [4N + 1][N + 1] (overwritten).  neg_h[r] bit x is
 * set when the bond (x, r)-(x+1 mod Lx, r) has J = -1, neg_v[r] bit x when
 * (x, r)-(x, r+1 mod Ly) has; either may be NULL (all J = 1).  Needs
 * Lx, Ly >= 3 (a side of 2 doubles bonds; the row pass above would count a
 * doubled bond once) and N <= 40. */
int oracle_row_words(int Lx, int Ly, const uint64_t *neg_h, const uint64_t *neg_v, uint64_t first,
                     uint64_t count, int n_threads, uint64_t *g) {
  if (Lx < 3 || Ly < 3 || Lx * Ly > 40 || n_threads < 1 || !g) return -1;
  const int N = Lx * Ly;
  const size_t cells = (size_t)(4 * N + 1) * (size_t)(N + 1);
  if (first > (1ull << N) || count > (1ull << N) - first) return -1;
  uint64_t nh[64] = {0}, nv[64] = {0};
  for (int r = 0; r < Ly; ++r) {
    nh[r] = neg_h ? neg_h[r] : 0;
    nv[r] = neg_v ? neg_v[r] : 0;
  }
  const uint64_t total = count;
  if ((uint64_t)n_threads > total) n_threads = total ? (int)total : 1;
  words_job *jobs = (words_job *)calloc((size_t)n_threads, sizeof(words_job));
  pthread_t *th = (pthread_t *)calloc((size_t)n_threads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -4; }
  int rc = 0, made = 0;
  for (int t = 0; t < n_threads; ++t) {
    jobs[t] = (words_job){Lx, Ly, first + total / (uint64_t)n_threads * (uint64_t)t,
                          first + (t == n_threads - 1 ? total : total / (uint64_t)n_threads * (uint64_t)(t + 1)),
                          nh, nv, (uint64_t *)calloc(cells, sizeof(uint64_t))};
    if (!jobs[t].table) { rc = -4; break; }
    made = t + 1;
  }
  if (rc == 0) {
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, words_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    memset(g, 0, cells * sizeof(uint64_t));
    for (int t = 0; t < n_threads; ++t)
      for (size_t k = 0; k < cells; ++k) g[k] += jobs[t].table[k];
  }
  for (int t = 0; t < made; ++t) free(jobs[t].table);
  free(jobs); free(th);
  return rc;
}
