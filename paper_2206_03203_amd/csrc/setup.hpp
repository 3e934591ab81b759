// Host-side setup of the solver: block split of eq. (4), approximate Schur
// complement of eq. (7) and smoothed-aggregation AMG hierarchies (Section 3.3).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "host_csr.hpp"
#include "mdp.h"

namespace mdp {

struct AmgParams {
  double theta = 0.02;
  int32_t max_coarse = 400;
  int32_t max_dense = 2000;
  int32_t max_levels = 10;
};

struct HLevel {
  HCsr A;                    // level operator
  HCsr P, R;                 // prolongator to this level from the next, R = P^T (not on the coarsest)
  HCsr Rf;                   // R (I - A D^-1) when applying it beats the residual and R (else 0 x 0)
  std::vector<double> dl1;   // l1 row norms sum_j |a_ij| (smoother diagonal)
  std::vector<int32_t> agg;  // aggregate per node (-1 = none); empty on the coarsest
};

struct HHier {
  std::vector<HLevel> lv;
  bool dense = false;               // coarsest solved with a dense inverse
  std::vector<double> coarse_inv;   // n_c x n_c row-major inverse when dense
  // Dense tail (derived at upload, not part of the hierarchy itself): the
  // V-cycle from level `tail` down is one linear operator of b, kept here as
  // an n_tail x n_tail row-major matrix and applied in place of those levels
  // (-1: none).  It was formed for the sweep counts and size bound below.
  int32_t tail = -1;
  int tail_pre = 0, tail_post = 0, tail_max = 0;
  std::vector<double> tail_op;
  int32_t n() const { return lv.empty() ? 0 : lv[0].A.nr; }
  // levels the device runs, whether the last is a dense product, and its
  // matrix, with the tail in use or not
  size_t depth(bool with_tail) const { return with_tail && tail >= 0 ? static_cast<size_t>(tail) + 1 : lv.size(); }
  bool ends_dense(bool with_tail) const { return (with_tail && tail >= 0) || dense; }
  const std::vector<double> &coarse_op(bool with_tail) const {
    return with_tail && tail >= 0 ? tail_op : coarse_inv;
  }
};

struct HostSystem {
  int32_t n = 0, n_o = 0, n_g = 0;
  std::vector<int32_t> perm;  // new index -> caller index ([Omega; Gamma], stable)
  bool identity = true;
  HCsr A;                     // full matrix in [Omega; Gamma] order, sorted rows
  HCsr Aoo, Aog, Ago, Agg;    // blocks of eq. (4)
  HCsr S;                     // S~ of eq. (7)
  HHier Ho, Hg;               // hierarchies on S~ and A_GG
  bool symmetric = true;
};

// Error carrying an MDP_* code.
struct SetupError {
  int code;
  std::string msg;
};

// Build everything on the host.  label (may be NULL): one label per unknown
// (the dimension of its subdomain) for dimension-aware aggregation on the
// finest level of each hierarchy.  Throws SetupError.
void build_host_system(const mdp_csr *A, const int32_t *part, const mdp_options &opt,
                       HostSystem &out, const int32_t *label = nullptr);

// Write / read the complete host setup (hierarchy file).  `amg` receives the
// AMG options the file was built with.  Both throw SetupError (MDP_EINVAL).
void save_host_system(const HostSystem &s, const mdp_options &o, const char *path);
void load_host_system(const char *path, HostSystem &out, mdp_options &amg);

// SA-AMG setup on one block (exposed for testing through the C ABI).
HHier amg_setup(const HCsr &A, const AmgParams &prm, const int32_t *labels = nullptr);

// Form h's dense tail for l1-Jacobi V-cycles with `pre` / `post` sweeps: the
// first level l >= 1 above the coarsest with at most max_n unknowns, when the
// coarsest level is dense; else clear it.  Does nothing when the tail was
// already formed for these arguments.
void form_tail(HHier &h, int pre, int post, int32_t max_n);
void clear_tail(HHier &h);

}  // namespace mdp
