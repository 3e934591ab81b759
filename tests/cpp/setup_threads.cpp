// Race check of the multithreaded host setup, built with ThreadSanitizer.
// For every host system named on the command line (hierarchy files written
// by the library) it runs the whole setup again (block split, S~ of eq. (7),
// both SA-AMG hierarchies of Section 3.3) on the stored matrix with the
// worker threads the environment sets, and requires the result to equal the
// stored setup bit for bit: the chunked parallel loops write disjoint rows
// and their results do not depend on the thread count.  Prints
// "failures: N" and exits with status 1 when N > 0 (ThreadSanitizer reports
// races on its own and fails the run).
#include <cstdio>
#include <cstring>
#include <vector>

#include "setup.hpp"

using namespace mdp;

static int fails = 0;

static bool same_csr(const HCsr &a, const HCsr &b) {
  return a.nr == b.nr && a.nc == b.nc && a.ptr == b.ptr && a.col == b.col &&
         (a.val.empty() || std::memcmp(a.val.data(), b.val.data(), a.val.size() * sizeof(double)) == 0) &&
         a.val.size() == b.val.size();
}

static void compare(const char *what, const HHier &a, const HHier &b) {
  if (a.lv.size() != b.lv.size() || a.dense != b.dense || a.coarse_inv != b.coarse_inv) {
    std::printf("FAIL %s: %zu vs %zu levels\n", what, a.lv.size(), b.lv.size());
    ++fails;
    return;
  }
  for (size_t l = 0; l < a.lv.size(); ++l) {
    const HLevel &x = a.lv[l], &y = b.lv[l];
    const bool ok = same_csr(x.A, y.A) && same_csr(x.P, y.P) && same_csr(x.R, y.R) && same_csr(x.Rf, y.Rf) &&
                    x.dl1 == y.dl1 && x.agg == y.agg;
    if (!ok) {
      std::printf("FAIL %s level %zu differs\n", what, l);
      ++fails;
    }
  }
}

int main(int argc, char **argv) {
  for (int a = 1; a < argc; ++a) {
    HostSystem s;
    mdp_options o{};
    load_host_system(argv[a], s, o);
    // the stored matrix is already in [Omega; Gamma] order: Omega first
    std::vector<int32_t> part(static_cast<size_t>(s.n), 0);
    for (int32_t i = s.n_o; i < s.n; ++i) part[i] = 1;
    mdp_csr c{};
    c.n = s.A.nr;
    c.nnz = s.A.nnz();
    c.row_ptr = s.A.ptr.data();
    c.col = s.A.col.data();
    c.val = s.A.val.data();
    HostSystem t;
    build_host_system(&c, part.data(), o, t);
    std::printf("== %s: n=%d n_o=%d n_g=%d, %zu + %zu levels\n", argv[a], s.n, s.n_o, s.n_g, t.Ho.lv.size(),
                t.Hg.lv.size());
    if (!same_csr(s.S, t.S)) {
      std::printf("FAIL S~ differs\n");
      ++fails;
    }
    compare("Omega hierarchy", s.Ho, t.Ho);
    compare("Gamma hierarchy", s.Hg, t.Hg);
  }
  std::printf("failures: %d\n", fails);
  return fails ? 1 : 0;
}
