/* Test driver: run the oracle's counts on one lattice read from stdin and
 * print the nonzero bins, so the same C code can be checked under the
 * address, undefined-behaviour and thread sanitizers (host code only).
 *
 * stdin: n nb then nb lines "i j J"; stdout: "E n_up count" per nonzero bin
 * of the brute force over all configurations (2 threads), then the same for
 * a split of the range into two halves and of the banded count (any
 * disagreement prints "mismatch"), then "bond b E n_up count" for the
 * bond-resolved counts. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_count_range(int n, int nb, const int32_t *bi, const int32_t *bj, const int32_t *bJ, uint64_t first,
                       uint64_t count, int n_threads, uint64_t *g);
int oracle_bond_split(int n, int nb, const int32_t *bi, const int32_t *bj, const int32_t *bJ, int n_threads,
                      uint64_t *g, uint64_t *gp);
int oracle_band_count(int n, int nb, const int32_t *bi, const int32_t *bj, const int32_t *bJ, uint64_t *g);

int main(void) {
  int n, nb;
  if (scanf("%d %d", &n, &nb) != 2 || n < 1 || n > 24 || nb < 0) return 2;
  int32_t *bi = calloc((size_t)nb + 1, 4), *bj = calloc((size_t)nb + 1, 4), *bJ = calloc((size_t)nb + 1, 4);
  for (int b = 0; b < nb; ++b)
    if (scanf("%d %d %d", &bi[b], &bj[b], &bJ[b]) != 3) return 2;
  int64_t S = 0;
  for (int b = 0; b < nb; ++b) S += bJ[b] < 0 ? -bJ[b] : bJ[b];
  const size_t cells = (size_t)(2 * S + 1) * (size_t)(n + 1);
  uint64_t *g = calloc(cells, 8), *h = calloc(cells, 8), *g2 = calloc(cells, 8), *gb = calloc(cells, 8);
  uint64_t *gp = calloc(cells * (size_t)(nb > 0 ? nb : 1), 8);
  const uint64_t total = (uint64_t)1 << n;
  if (oracle_count_range(n, nb, bi, bj, bJ, 0, total, 2, g)) return 3;
  if (oracle_count_range(n, nb, bi, bj, bJ, 0, total / 3, 3, h)) return 3;
  if (oracle_count_range(n, nb, bi, bj, bJ, total / 3, total - total / 3, 2, h)) return 3;
  if (oracle_bond_split(n, nb, bi, bj, bJ, 3, g2, gp)) return 3;
  const int band = oracle_band_count(n, nb, bi, bj, bJ, gb);   /* -2, -3: too wide, not run */
  if (band != 0 && band != -2 && band != -3) return 3;
  for (size_t c = 0; c < cells; ++c)
    if (g[c]) printf("%lld %d %llu\n", (long long)(c / (size_t)(n + 1)) - (long long)S, (int)(c % (size_t)(n + 1)),
                     (unsigned long long)g[c]);
  printf("split\n");
  for (size_t c = 0; c < cells; ++c)
    if (h[c] != g[c] || g2[c] != g[c] || (band == 0 && gb[c] != g[c])) printf("mismatch %zu\n", c);
  for (int b = 0; b < nb; ++b)
    for (size_t c = 0; c < cells; ++c)
      if (gp[(size_t)b * cells + c])
        printf("bond %d %lld %d %llu\n", b, (long long)(c / (size_t)(n + 1)) - (long long)S,
               (int)(c % (size_t)(n + 1)), (unsigned long long)gp[(size_t)b * cells + c]);
  free(bi); free(bj); free(bJ); free(g); free(h); free(g2); free(gb); free(gp);
  return 0;
}
