// Device-resident solver state: the uploaded matrices and AMG hierarchies,
// the Krylov workspace and the FGMRES driver.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "types.hpp"
#include "runtime.hpp"
#include "setup.hpp"

namespace mdp {

// A device sparse matrix, stored either as CSR (long rows; `lpr` lanes per
// row) or as sliced ELL with 64-row slices (`sell`; `ptr` then holds the
// slice offsets).
template <typename T>
struct DCsr {
  int32_t nr = 0, nc = 0;
  int64_t nnz = 0;
  int lpr = 8;
  bool sell = false;
  bool scalar = false;  // CSR, one thread per row
  int32_t nslices = 0;
  DevMem ptr, col, val;
  const int *p() const { return dptr<const int>(ptr); }
  const int *c() const { return dptr<const int>(col); }
  const T *v() const { return dptr<const T>(val); }
};

template <typename T>
struct DLevel {
  int32_t n = 0;
  DCsr<T> A, P, R;
  DevMem dinv;     // 1 / sum_j |a_ij|
  DevMem x, b, t;  // coarse-level unknown / right-hand side, smoothing scratch
  DevMem r;        // residual after pre-smoothing
};

template <typename T>
struct DHier {
  std::vector<DLevel<T>> lv;
  bool dense = false;
  int32_t nc = 0;
  DevMem cinv;           // dense FP64 inverse of the coarsest level
  DevMem tmp_res, tmp_dz;  // extra cycles: residual and correction at level 0
  DevMem tmp_pp;          // coarsest l1-Jacobi ping-pong
  bool is_omega = false;  // hierarchy on S~ (its finest level is timed separately)
  int32_t n() const { return lv.empty() ? 0 : lv[0].n; }
};

// Preconditioner M_L in precision T (Algorithm 1).
template <typename T>
struct Precond {
  DHier<T> Ho, Hg;
  DCsr<T> Ago;
  DevMem rg;  // r_Gamma - A_GO z_Omega
  int32_t n_o = 0, n_g = 0;
  int vcycles = 1;
};

struct Workspace {
  int64_t ld = 0;  // leading dimension of V / Z columns
  int m = 0;       // restart length
  DevMem V, Z, w, w2, bp, xp, rin;
  DevMem Hr, cs, sn, g, y, hist, hprev, coef, sums;
  DevMem partial, npartial, scalar;  // reduction scratch
  DevMem state;                      // GmresState
  GmresState *host_state = nullptr;  // pinned, one slot per Arnoldi step
  double *host_scalar = nullptr;     // pinned
  std::vector<hipEvent_t> ev;
  ~Workspace();
};

struct Solver {
  HostSystem host;
  mdp_options opt{};
  bool on_device = false;
  int32_t n = 0, n_o = 0, n_g = 0;
  DCsr<double> A;  // full matrix, [Omega; Gamma] order
  DevMem perm;     // new -> caller index
  std::unique_ptr<Precond<double>> pc64;
  std::unique_ptr<Precond<float>> pc32;
  Workspace ws;
  double setup_ms = 0.0;

  void upload(hipStream_t s);
  int solve(const double *b, double *x, hipStream_t s, mdp_stats *st);
  void apply(int op, const double *x, double *y, hipStream_t s);
};

}  // namespace mdp

struct mdp_handle {
  mdp::Solver s;
};
