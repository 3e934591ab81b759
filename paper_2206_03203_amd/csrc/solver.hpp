// Device-resident solver state: uploaded matrices and AMG hierarchies, the
// Krylov workspace, and the FGMRES driver shared by single and batched solves.
//
// A "pair" is one (system, right-hand side) whose Krylov process runs on its
// own; a single solve is a batch of one pair.  Several systems are solved
// together as one block-diagonal system whose unknowns are laid out as
// [Omega of every pair; Gamma of every pair], so that every sparse kernel of
// the single-system path applies unchanged.
#pragma once

#include <hip/hip_runtime.h>

#include <memory>
#include <vector>

#include "runtime.hpp"
#include "setup.hpp"
#include "types.hpp"

namespace mdp {

// A device sparse matrix: diagonal storage (`dia`, `ptr` = the ndiag
// offsets, `val` = ndiag x nr), diagonals plus a CSR remainder (`hyb`: the
// ndiag offsets in `doff`, their values ndiag x nr in `dval`, the remaining
// rem_nnz entries in ptr / col / val), sliced ELL (`sell`, 64-row slices,
// `ptr` = slice offsets), CSR with one thread per row (`scalar`), or CSR with
// `lpr` lanes per row and `batch` entries in flight per lane.
template <typename T>
struct DCsr {
  int32_t nr = 0, nc = 0;
  int64_t nnz = 0;
  int lpr = 8;
  int batch = 4;  // CSR-vector: entries in flight per lane
  bool dia = false;
  bool hyb = false;
  int32_t ndiag = 0;
  int64_t rem_nnz = 0;
  int32_t split = 0;  // diagonals + remainder: rows [split, nr) are dispatched first
  DevMem doff, dval;
  bool sell = false;
  bool scalar = false;
  int32_t nslices = 0;
  DevMem ptr, col, val;
  const int *rowpair = nullptr;  // batched: system (kb > 1) or pair (kb = 1) of each row, not owned; else NULL
  // Vector blocks: kb right-hand-side blocks share each matrix read; block r
  // of x starts r * bxs further on, block r of b, dinv, y, y2 r * bys further.
  int kb = 1;
  int64_t bxs = 0, bys = 0;
  int nsys = 1;  // systems per block (pair of row i in block r: r * nsys + rowpair[i])
  const int *p() const { return dptr<const int>(ptr); }
  const int *rp() const { return rowpair; }
  const int *c() const { return dptr<const int>(col); }
  const T *v() const { return dptr<const T>(val); }
};

// One level of a (possibly batched) hierarchy.  Rows [0, ncont) belong to
// systems that continue to the next level; then come the systems whose
// coarsest level this is: dense-inverse ones, then l1-Jacobi-swept ones
// (rows [sw_off, n)).
template <typename T>
struct DLevel {
  int32_t n = 0;
  int32_t ncont = 0;
  DCsr<T> A, P, R;  // A: operator of the continuing systems; P, R to/from the next level
  bool fused = false;  // R holds R (I - A D^-1) and restricts b directly (no residual product)
  DevMem dinv;      // n entries: 1 / sum_j |a_ij|
  int32_t ndense = 0, max_dense_n = 0;
  DevMem dense;     // DenseDesc[ndense]
  int32_t sw_off = 0;
  DCsr<T> Asw;      // swept coarsest systems, indices relative to sw_off
  bool sw_diag = false;  // every swept system is diagonal: D^-1 b solves it
  DevMem x, b, t, r;  // unknown, right-hand side, smoothing iterate, residual (and sweep ping-pong)
  DevMem pp;          // ping-pong for the swept coarsest systems
  // multicolour Gauss-Seidel (MDP_SMOOTH_GS): the continuing systems'
  // operator in plain CSR, its rows grouped by colour, and 1 / a_ii
  DCsr<T> Ag;
  DevMem gs_rows, dg;
  std::vector<int32_t> gs_off;  // colour c: gs_rows[gs_off[c] .. gs_off[c + 1])
  std::vector<int64_t> gs_nnz;  // entries in the rows of each colour
  int gs_lpr = 1;               // lanes per row of the sweep kernel
};

// With kb > 1 (several right-hand sides per system in a batch) every level
// vector holds kb blocks of the one-copy layout: block r is right-hand side r
// of every system, and n, ncont and sw_off count one block.  The matrices are
// stored once and applied to all blocks in one pass.
template <typename T>
struct DHier {
  std::vector<DLevel<T>> lv;
  int kb = 1;
  int pre = 1, post = 1;        // smoothing sweeps before and after the coarse correction
  bool gs = false;              // multicolour Gauss-Seidel instead of l1-Jacobi
  std::vector<DevMem> rowpair;  // batched: per level, the pair of each row
  DevMem cinv;            // dense FP64 inverses of the coarsest levels
  DevMem tmp_res, tmp_dz; // extra cycles: residual and correction at level 0
  bool is_omega = false;  // hierarchy on S~ (its finest level is timed separately)
  int32_t n() const { return lv.empty() ? 0 : lv[0].n; }  // one block
  int64_t nfull() const { return static_cast<int64_t>(kb) * n(); }
  // true when nothing at level 0 smooths (only dense-solved systems there)
  bool dense_only() const { return lv.size() == 1 && lv[0].ncont == 0 && lv[0].sw_off == lv[0].n; }
};

// Block preconditioner in precision T: M_L (Algorithm 1), M_D or M_U.
template <typename T>
struct Precond {
  DHier<T> Ho, Hg;
  DCsr<T> Ago;  // A_GO (lower form)
  DCsr<T> Aog;  // A_OG (upper form)
  DevMem rg;    // r_Gamma - A_GO z_Omega (lower); r_Omega - A_OG z_Gamma (upper)
  int32_t n_o = 0, n_g = 0;  // all blocks
  int vcycles = 1;
  int form = MDP_BLOCK_LOWER;
};

// Tile work list over the pairs' unknowns (global vector layout).
struct Layout {
  int npairs = 0;
  int64_t n = 0;
  int ntiles = 0;
  DevMem tiles;     // Tile[ntiles], grouped by pair
  DevMem tile_off;  // npairs + 1
  std::vector<int64_t> rows;  // unknowns per pair (host)
  // ranges[p] = the (start, length) pieces of pair p in the global vector
  void build(const std::vector<std::vector<std::pair<int64_t, int64_t>>> &ranges, int64_t n_total,
             hipStream_t s);
};

// Arnoldi steps replayed from captured HIP graphs (MDP_GRAPHS): exec[j] for
// step j, exec[m + 1 + j] for a cycle's last step j (which reuses the
// preconditioned column j - 1).  A graph holds the addresses of the
// workspace and of the solve's matrices, so it is valid for the workspace
// `ws` it was captured with and for the life of its owner.
struct StepGraphs {
  std::vector<hipGraphExec_t> exec;
  const void *ws = nullptr;
  uint64_t ws_gen = 0;  // the workspace's generation at capture
  bool failed = false;  // capture or instantiation failed once: launch directly
  void clear();
  ~StepGraphs() { clear(); }
};

struct Workspace {
  int64_t ld = 0;  // leading dimension of V / Z columns
  int m = 0;       // restart length
  int npairs = 0;   // pairs the per-pair arrays hold
  int ntiles = 0;   // tiles the per-tile partial sums hold
  int ldv = 0;     // per-pair stride of length-(m+1) arrays
  int sstride = 0; // per-pair stride of the step sums
  size_t tsz = 0;   // bytes per entry of Z and rin (4: FP32 preconditioner, 8: FP64)
  uint64_t gen = 0; // changes whenever the device arrays move (graphs hold their addresses)
  DevMem V, Z, w, rin, bp, xp;
  DevMem Hr, cs, sn, g, y, hist, hprev, coef, sums;
  DevMem partial, npart;
  DevMem state, ctl, kmaxp, tolp, scale0, active, norms;  // scale0: per pair, 1 / beta of the cycle (mixed)
  BatchCtl *host_ctl = nullptr;      // pinned, one slot per step
  BatchCtl *host_ctl_dev = nullptr;  // its device address
  GmresState *host_state = nullptr;  // pinned, npairs
  double *host_norms = nullptr;      // pinned, npairs
  double *host_hist = nullptr;       // pinned, m: a cycle's residual estimates (single-pair solves)
  std::vector<double> history;       // |g_{k+1}| / ||b|| per iteration of the last single-pair solve
  std::vector<hipEvent_t> ev;
  StepGraphs graphs;               // single-system solves on this workspace (MDP_GRAPHS)
  StepGraphs graphs64;             // the FP64 re-solves of MDP_FALLBACK_FP64 on it
  hipStream_t own = nullptr;       // non-blocking stream for solves handed the legacy stream
  hipEvent_t handoff = nullptr;
  hipStream_t own_stream();        // created on first use
  void alloc(int64_t n, int m, int npairs, int ntiles, size_t tsz, hipStream_t s);
  // device bytes alloc() takes for these sizes (with bp / xp when `perm`)
  static size_t bytes_for(int64_t n, int m, int npairs, int ntiles, size_t tsz, bool perm);
  // holds at least these sizes (and bp / xp)
  bool fits(int64_t n, int m, int npairs, int ntiles, size_t tsz) const;
  void release();           // free everything (alloc may be called again)
  size_t device_bytes() const;
  bool allocated() const { return V.get() != nullptr; }
  ~Workspace() { release(); }
};

struct PairIO {
  const double *b;  // caller's right-hand side (caller order), device
  double *x;        // caller's solution (caller order), device
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
  Layout layout;
  Workspace ws;
  double setup_ms = 0.0;

  void upload(hipStream_t s);
  void ensure_workspace(hipStream_t s);  // (re)allocate the Krylov workspace if released
  size_t workspace_bytes_needed() const;
  // fp64_only: solve from zero with the FP64 preconditioner at once (the
  // fallback of a mixed column whose four-column solve failed)
  int solve(const double *b, double *x, hipStream_t s, mdp_stats *st, bool fp64_only = false);
  // MDP_FALLBACK_FP64: the FP64 preconditioner (built from the kept host
  // hierarchy) and a workspace wide enough for FP64 directions
  void ensure_fp64(hipStream_t s);
  void apply(int op, const double *x, double *y, hipStream_t s);
  // The launches of apply, without allocation or synchronisation; in mixed
  // precision `in` and `out` stage the FP32 copies of x and y (n entries each)
  void enqueue_apply(int op, const double *x, double *y, hipStream_t s, float *in, float *out);
};

// A block-diagonal batch of pairs (a system appears once per right-hand side).
// When every system of the batch has kMultiRhs right-hand sides, the pairs
// run in right-hand-side-major order (pair r * nsys + s is right-hand side r
// of system s) and the preconditioner's matrices are stored once for all
// right-hand sides (kb = kMultiRhs); otherwise each pair is its own block.
struct Batch {
  std::vector<const Solver *> sys;  // per pair, caller's order
  int npairs = 0;
  int kb = 1, nsys = 0;    // blocks, and systems per block
  std::vector<int> order;  // internal pair -> caller's pair
  int32_t n = 0, n_o = 0, n_g = 0;
  mdp_options opt{};
  DCsr<double> A;
  DevMem gidx;  // per global row: caller index within its pair's system
  DevMem gpair; // per global row: internal pair (also the row-to-pair map of A)
  std::unique_ptr<Precond<double>> pc64;
  std::unique_ptr<Precond<float>> pc32;
  Layout layout;
  Workspace ws;              // own workspace (left empty when `wsp` is set)
  Workspace *wsp = nullptr;  // shared workspace of at least this batch's sizes
  StepGraphs graphs;         // this batch's Arnoldi steps (MDP_GRAPHS)
  // alloc_ws = false: leave the workspace to the caller (set wsp before solve)
  void build(const std::vector<const Solver *> &pairs, hipStream_t s, bool alloc_ws = true);
  int solve(const std::vector<PairIO> &io, hipStream_t s, mdp_stats *st);
};

// Record the autotuner's choices in the text file `path` and use the ones
// already recorded there (NULL: stop recording).
void set_tune_file(const char *path);

}  // namespace mdp

struct mdp_handle;

namespace mdp {

// Solve the columns of one system (st: one entry per column), four at a
// time through the handle's four-column batch when `group` is set and the
// batch fits its budget, the rest one by one; returns the most severe code.
// After an error the columns not solved carry that code.  *grouped (may be
// NULL) counts the columns solved four at a time.
int solve_columns(mdp_handle *h, const std::vector<PairIO> &cols, hipStream_t s, mdp_stats *st, bool group,
                  int64_t *grouped = nullptr);

}  // namespace mdp

struct mdp_handle {
  mdp::Solver s;
  // mdp_solve with four or more columns: the same system as a batch of
  // kMultiRhs pairs sharing the preconditioner's matrix reads (built on first
  // use when the process-wide budget for such plans has room, kept until
  // mdp_destroy)
  std::unique_ptr<mdp::Batch> rhs4;  // its Krylov workspace is the device's shared one
  int rhs4_dev = 0;        // the device the plan was built on
  int64_t rhs4_bytes = 0;  // device bytes the plan holds (counted in the budget)
  int64_t rhs4_need = 0;   // a plan that did not fit: its size (retried when the budget has room)
  bool rhs4_failed = false;  // the device ran out of memory building it: one column at a time
};
