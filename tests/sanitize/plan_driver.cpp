// Test driver: the library's host-side planner (plan.cpp, bond_plan.cpp)
// built with g++ so that the address, undefined-behaviour and leak
// sanitizers can watch it.  For every lattice read from stdin it creates the
// plan under several tunes and prints the layout, the histogram shape and the
// backward workspace, which the test compares with the library's answers.
//
// stdin: lattices "n nb" then nb lines "i j J", repeated to EOF.
// The device-side pieces a host-only plan never reaches (freeing device
// copies, which are never made here) are replaced by host definitions.
#include <cstdio>
#include <vector>

#include "../../paper_1110_2561_amd/csrc/bond.h"
#include "../../paper_1110_2561_amd/csrc/internal.h"

namespace ising {
void bond_plan_free(BondPlan *b) { delete b; }
}  // namespace ising

extern "C" ising_status ising_plan_destroy(ising_plan *p) {
  if (!p) return ISING_OK;
  ising::bond_plan_free(p->bond);
  delete p;
  return ISING_OK;
}

int main() {
  int n, nb, id = 0;
  const ising_tune tunes[] = {{0, 0, 0, 0, 0, 0}, {0, 3, 4, 0, 0, 0}, {0, 0, 0, 4, 0, 0}, {0, 0, 0, 0, 0, 5},
                              {12, 8, 0, 0, 0, 0}};
  while (std::scanf("%d %d", &n, &nb) == 2) {
    std::vector<int32_t> bi(nb), bj(nb), bJ(nb);
    for (int b = 0; b < nb; ++b)
      if (std::scanf("%d %d %d", &bi[b], &bj[b], &bJ[b]) != 3) return 2;
    const ising_lattice lat{n, nb, bi.data(), bj.data(), bJ.data()};
    for (int t = 0; t < 5; ++t) {
      ising_plan *p = nullptr;
      const ising_status st = ising_plan_create(&lat, &tunes[t], &p);
      std::printf("lattice %d tune %d status %d", id, t, int(st));
      if (st == ISING_OK) {
        int32_t n_e, n_m, e_min, k, j;
        uint64_t chunks;
        std::vector<int32_t> bos(n);
        ising_hist_shape(p, &n_e, &n_m, &e_min);
        ising_plan_layout(p, bos.data(), &k, &j, &chunks);
        size_t ws = 0;
        const ising_status wst = ising_bond_workspace(p, &ws);
        std::printf(" shape %d %d %d inner %d tile %d chunks %llu ws %d %zu bits", n_e, n_m, e_min, k, j,
                    (unsigned long long)chunks, int(wst), ws);
        for (int s = 0; s < n; ++s) std::printf(" %d", bos[s]);
        ising_plan_destroy(p);
      }
      std::printf("\n");
    }
    ++id;
  }
  return 0;
}
