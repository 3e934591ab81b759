// Writes the dense V-cycle tails that form_tail (csrc/setup.cpp) builds for
// the two hierarchies of each host system named on the command line
// (hierarchy files written by the library), for the CPU test that compares
// them with the oracle's V-cycle started at the same level.
//   tail_check PRE POST MAX_N OUT FILE...
// OUT holds, per system and hierarchy (Omega, then Gamma): int32 level
// (-1: none), int32 n, then n * n doubles (row-major) when level >= 0.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "setup.hpp"

using namespace mdp;

int main(int argc, char **argv) {
  if (argc < 6) {
    std::fprintf(stderr, "usage: tail_check PRE POST MAX_N OUT FILE...\n");
    return 2;
  }
  const int pre = std::atoi(argv[1]), post = std::atoi(argv[2]);
  const int32_t max_n = std::atoi(argv[3]);
  FILE *out = std::fopen(argv[4], "wb");
  if (!out) return 2;
  for (int a = 5; a < argc; ++a) {
    HostSystem s;
    mdp_options o{};
    load_host_system(argv[a], s, o);
    for (HHier *h : {&s.Ho, &s.Hg}) {
      form_tail(*h, pre, post, max_n);
      const int32_t l = h->tail;
      const int32_t n = l >= 0 ? h->lv[l].A.nr : 0;
      std::fwrite(&l, sizeof l, 1, out);
      std::fwrite(&n, sizeof n, 1, out);
      if (l >= 0) std::fwrite(h->tail_op.data(), sizeof(double), h->tail_op.size(), out);
      std::printf("%s: hierarchy of %zu levels, tail at level %d (n = %d)\n", argv[a], h->lv.size(), l, n);
    }
  }
  std::fclose(out);
  return 0;
}
