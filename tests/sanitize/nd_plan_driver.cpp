// Host driver for an AddressSanitizer / UndefinedBehaviorSanitizer build of
// the nested-dissection planner (paper_2408_03571_amd/csrc/nd_plan.cpp), the
// host code that lays out the coarse solver's fronts (Sec. 3: exact coarse
// solve of A_0 = R_0 A R_0^T).  Built by tests/test_sanitize.py with the
// host compiler only (no device code); each argument quadruple
// ncx,ncy,reach,leaf is planned and, when check=1, structurally checked.
//   usage: nd_plan_driver ncx ncy reach leaf check [ncx ncy reach leaf check ...]
#include <cstdio>
#include <cstdlib>
#include <string>

#include "hs_internal.h"

namespace hs {
void set_error(const std::string& m) { std::fprintf(stderr, "%s\n", m.c_str()); }
}  // namespace hs

int main(int argc, char** argv) {
  if (argc < 6 || (argc - 1) % 5 != 0) {
    std::fprintf(stderr, "usage: %s ncx ncy reach leaf check ...\n", argv[0]);
    return 2;
  }
  int bad = 0;
  for (int a = 1; a + 4 < argc; a += 5) {
    const int ncx = std::atoi(argv[a]), ncy = std::atoi(argv[a + 1]);
    const int reach = std::atoi(argv[a + 2]), leaf = std::atoi(argv[a + 3]), check = std::atoi(argv[a + 4]);
    if (check) {
      int64_t st[8] = {};
      const hs_status s = hs_nd_plan_check(ncx, ncy, reach, leaf, st);
      std::printf("check %d x %d reach %d leaf %d: status %d, %lld fronts, %lld levels\n", ncx, ncy, reach, leaf,
                  (int)s, (long long)st[0], (long long)st[1]);
      bad |= (s != HS_OK);
    } else {
      const hs::NDPlan p = hs::build_nd_plan(ncx, ncy, reach, leaf);
      std::printf("plan %d x %d reach %d leaf %d: %zu fronts, g %lld, v %lld\n", ncx, ncy, reach, leaf,
                  p.fronts.size(), (long long)p.g_elems, (long long)p.v_elems);
    }
  }
  return bad;
}
