// Constants and device-visible structs shared by host and kernel code.
#pragma once

#include <cstdint>

namespace mdp {

constexpr int kThreads = 256;
constexpr int kXcds = 8;
constexpr int kMaxCols = 64;      // Krylov basis columns handled by one Arnoldi pass
constexpr int kCsrBatch = 4;       // CSR-vector entries in flight per lane under the fixed rule
constexpr int kMaxDiag = 16;       // most offsets of the diagonal layouts
constexpr int kMultiRhs = 4;       // right-hand sides that share one matrix read in a batch
constexpr int kMaxSweeps = 8;      // l1-Jacobi sweeps before / after the coarse correction, at most
constexpr int kDotU = 9;          // elements per thread in the Arnoldi passes (tiles of up to 2304)
constexpr int kTileElems = 256 * kDotU;

// Per-cycle FGMRES state in device memory.
struct GmresState {
  int done;        // the cycle has ended: every later kernel of the cycle returns at once
  int skip_apply;  // no further preconditioner / system-matrix applications this cycle
  int finishing;   // the next step only finalises the last Hessenberg column
  int k;           // Krylov basis size whose least-squares problem is final
  int nan;         // a non-finite value appeared
  int pad;
  double est;      // |g_k|: residual-norm estimate for the final basis of size k
  double nu;       // scale applied to the provisional vector of the next step
};

// Batch-wide control words (device memory), reset at the start of a cycle.
struct BatchCtl {
  int napply_left;     // pairs still applying the preconditioner this cycle
  int ndone;           // pairs whose cycle has ended
  int skip_all_apply;  // set when napply_left reaches 0: whole-batch kernels return at once
  int all_done;        // set when ndone reaches the number of pairs
};

// What the update pass of step j also writes for step j + 1 (all fields may
// be NULL): the preconditioner input in mixed precision (FP32 copy of
// u_{j+1}, and D^-1 of it on the first n_o rows, the host block), or in FP64
// the first smoothing iterate D^-1 u_{j+1} on those rows; and the step's
// control word, copied to the host (device-visible pinned memory).
struct NextInput {
  float *rin;
  float *t32;
  const float *dinv32;
  double *t64;
  const double *dinv64;
  int64_t n_o;
  BatchCtl *host_ctl;
  const BatchCtl *ctl;
};

// A contiguous piece (at most kTileElems entries) of one (system, rhs) pair's
// unknowns in the global vector layout.
struct Tile {
  int64_t start;
  int32_t len;
  int32_t pair;
};

// Coarsest level of one system solved with its dense inverse.
struct DenseDesc {
  int32_t row;      // first row in the level vector
  int32_t n;        // size
  int64_t inv_off;  // offset of its row-major inverse in the concatenated store
};

// Per-step coefficients written by the finalise kernel for the update pass.
//   q_j     = (u_j - sum_i a_i q_i) * inv_r
//   u_{j+1} = (w - sum_i b_i q_i - hj q_j) * inv_nu
struct DcgsCoef {
  double inv_r, hj, inv_nu, pad;
  double a[kMaxCols + 1];
  double b[kMaxCols + 1];
};

}  // namespace mdp
