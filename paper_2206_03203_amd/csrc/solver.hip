// Device side of the solve phase: upload of the host-built hierarchy, the
// V-cycle that defines Q_OO / Q_GG (Section 3.3), the preconditioner action of
// Algorithm 1 (M_L of eq. (8)) and right-preconditioned flexible GMRES
// (Section 3.2; zero initial guess and relative-residual stop, Section 4).
//
// Precision: the preconditioner runs in T (double, or float in mixed mode);
// the outer matrix, Krylov basis V, Hessenberg/Givens data and the coarsest
// dense inverse are always FP64.  Z (the preconditioned directions) is kept
// in T: A z_j is formed from the stored z_j, so FP32 storage is exact for
// the flexible method.
//
// Arnoldi uses classical Gram-Schmidt applied twice (CGS2): every pass reads
// each basis vector once and reductions use fixed trees, so results do not
// depend on scheduling.  Basis vectors are stored unnormalised with a
// per-column scale (1/norm) applied on every read, which saves a pass.
#include <chrono>
#include <cmath>
#include <cstring>
#include <limits>
#include <type_traits>

#include "kernels.hpp"
#include "ktimer.hpp"
#include "solver.hpp"

namespace mdp {

namespace {

// Lanes per row for the CSR-vector kernel: enough that one batch of
// kCsrBatch entries per lane covers an average row.
int choose_lpr(int64_t nnz, int32_t nr) {
  const double avg = nr > 0 ? static_cast<double>(nnz) / nr : 0.0;
  int l = 4;
  while (l * kCsrBatch < avg && l < 64) l *= 2;
  return l;
}

template <typename T>
void upload_vec(DevMem &d, const std::vector<T> &h, hipStream_t s) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty()) MDP_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Sliced ELL pays off when rows are short and similar within 64-row slices.
template <typename T>
void upload_csr(const HCsr &h, DCsr<T> &d, hipStream_t s, std::vector<std::vector<T>> &keep) {
  d.nr = h.nr;
  d.nc = h.nc;
  d.nnz = h.nnz();
  d.lpr = choose_lpr(d.nnz, d.nr);
  const int32_t ns = (h.nr + 63) / 64;
  int64_t padded = 0;
  int32_t maxlen = 0;
  for (int32_t sl = 0; sl < ns; ++sl) {
    int32_t w = 0;
    for (int32_t r = sl * 64; r < std::min(h.nr, sl * 64 + 64); ++r) w = std::max(w, h.ptr[r + 1] - h.ptr[r]);
    padded += 64 * static_cast<int64_t>(w);
    maxlen = std::max(maxlen, w);
  }
  // sliced ELL when slices carry little padding; one thread per row for other
  // short rows; LPR lanes per row otherwise
  const double avg = h.nr > 0 ? static_cast<double>(d.nnz) / h.nr : 0.0;
  d.sell = h.nr > 0 && maxlen <= 64 && padded <= 23 * std::max<int64_t>(d.nnz, 1) / 20 &&
           padded < std::numeric_limits<int32_t>::max();
  d.scalar = !d.sell && avg <= 12.0;
  if (!d.sell) {
    upload_vec(d.ptr, h.ptr, s);
    upload_vec(d.col, h.col, s);
    keep.emplace_back(h.val.begin(), h.val.end());
    upload_vec(d.val, keep.back(), s);
    return;
  }
  d.nslices = ns;
  std::vector<int32_t> soff(static_cast<size_t>(ns) + 1, 0), col(static_cast<size_t>(padded));
  std::vector<T> val(static_cast<size_t>(padded), T(0));
  int64_t o = 0;
  for (int32_t sl = 0; sl < ns; ++sl) {
    const int32_t r0 = sl * 64, r1 = std::min(h.nr, r0 + 64);
    int32_t w = 0;
    for (int32_t r = r0; r < r1; ++r) w = std::max(w, h.ptr[r + 1] - h.ptr[r]);
    soff[sl] = static_cast<int32_t>(o);
    for (int32_t lane = 0; lane < 64; ++lane) {
      const int32_t r = r0 + lane;
      const int32_t len = r < r1 ? h.ptr[r + 1] - h.ptr[r] : 0;
      int32_t lastc = 0;
      for (int32_t k = 0; k < w; ++k) {
        const int64_t dst = o + static_cast<int64_t>(k) * 64 + lane;
        if (k < len) {
          lastc = h.col[h.ptr[r] + k];
          col[dst] = lastc;
          val[dst] = static_cast<T>(h.val[h.ptr[r] + k]);
        } else {
          col[dst] = lastc;  // padding: a valid, nearby column with value 0
        }
      }
    }
    o += static_cast<int64_t>(w) * 64;
  }
  soff[ns] = static_cast<int32_t>(o);
  upload_vec(d.ptr, soff, s);
  upload_vec(d.col, col, s);
  keep.push_back(std::move(val));
  upload_vec(d.val, keep.back(), s);
}

template <typename T>
void upload_hier(const HHier &h, DHier<T> &d, hipStream_t s, std::vector<std::vector<T>> &keep) {
  d.lv.clear();
  d.lv.resize(h.lv.size());
  for (size_t l = 0; l < h.lv.size(); ++l) {
    const HLevel &hl = h.lv[l];
    DLevel<T> &dl = d.lv[l];
    dl.n = hl.A.nr;
    upload_csr(hl.A, dl.A, s, keep);
    std::vector<T> dinv(hl.dl1.size());
    for (size_t i = 0; i < dinv.size(); ++i) dinv[i] = static_cast<T>(1.0 / hl.dl1[i]);
    keep.push_back(std::move(dinv));
    upload_vec(dl.dinv, keep.back(), s);
    const size_t nb = static_cast<size_t>(std::max(dl.n, 1)) * sizeof(T);
    dl.x.alloc(nb);
    dl.b.alloc(nb);
    dl.t.alloc(nb);
    dl.r.alloc(nb);
    if (l + 1 < h.lv.size()) {
      upload_csr(hl.P, dl.P, s, keep);
      upload_csr(hl.R, dl.R, s, keep);
    }
  }
  d.dense = h.dense;
  d.nc = h.lv.back().A.nr;
  if (h.dense) upload_vec(d.cinv, h.coarse_inv, s);
  const size_t n0 = static_cast<size_t>(std::max(d.n(), 1)) * sizeof(T);
  d.tmp_res.alloc(n0);
  d.tmp_dz.alloc(n0);
  d.tmp_pp.alloc(2 * static_cast<size_t>(std::max(d.nc, 1)) * sizeof(T));
}

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, 8192)));
}

// Algorithmic bytes of one sparse product: matrix values, column indices and
// row pointers once, each vector entry read or written once.
template <int MODE, typename TA, typename TX, typename TY>
double spmv_bytes(const DCsr<TA> &A) {
  double b = (sizeof(TA) + 4.0) * A.nnz + 4.0 * (A.nr + 1.0);
  const double sx = sizeof(TX), sy = sizeof(TY);
  if (MODE == kPlain) b += sx * A.nc + sy * A.nr;
  if (MODE == kResid) b += sx * A.nc + 2 * sy * A.nr;
  if (MODE == kSmooth) b += sx * A.nc + 3 * sy * A.nr;  // x, b, dinv, y
  if (MODE == kPre0) b += 2 * sy * A.nc + 2 * sy * A.nr;  // b, dinv; y2, y
  if (MODE == kAccum) b += sx * A.nc + 2 * sy * A.nr;
  if (MODE == kPlainScale) b += sx * A.nc + 2 * sy * A.nr;   // x; dinv, y (+ y2)
  if (MODE == kResidScale) b += sx * A.nc + 4 * sy * A.nr;   // x; b, dinv, y, y2
  if (MODE == kPlainScale) b += sy * A.nr;
  return b;
}

template <int LPR, int MODE, typename TA, typename TX, typename TY>
void spmv_launch(const DCsr<TA> &A, const TX *x, const TY *b, const TY *dinv, TY *y, TY *y2,
                 const int *gate, hipStream_t s, int kind) {
  const int64_t rows_per_blk = kThreads / LPR;
  const int blocks = static_cast<int>((A.nr + rows_per_blk - 1) / rows_per_blk);
  timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
    hipLaunchKernelGGL((spmv_kernel<LPR, MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr,
                       A.p(), A.c(), A.v(), x, b, dinv, y, y2, gate);
  });
}

template <int MODE, typename TA, typename TX, typename TY>
void spmv(const DCsr<TA> &A, const TX *x, const TY *b, const TY *dinv, TY *y, TY *y2, const int *gate,
          hipStream_t s, int kind = kKcOther) {
  if (A.nr == 0) return;
  if (A.sell) {
    const int blocks = (A.nslices + (kThreads / 64) - 1) / (kThreads / 64);
    timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
      hipLaunchKernelGGL((sell_kernel<MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr, A.nslices,
                         A.p(), A.c(), A.v(), x, b, dinv, y, y2, gate);
    });
    return;
  }
  if (A.scalar) {
    const int blocks = (A.nr + kThreads - 1) / kThreads;
    timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
      hipLaunchKernelGGL((csr_scalar_kernel<MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr, A.p(),
                         A.c(), A.v(), x, b, dinv, y, y2, gate);
    });
    return;
  }
  switch (A.lpr) {
    case 4: spmv_launch<4, MODE>(A, x, b, dinv, y, y2, gate, s, kind); break;
    case 8: spmv_launch<8, MODE>(A, x, b, dinv, y, y2, gate, s, kind); break;
    case 16: spmv_launch<16, MODE>(A, x, b, dinv, y, y2, gate, s, kind); break;
    case 32: spmv_launch<32, MODE>(A, x, b, dinv, y, y2, gate, s, kind); break;
    default: spmv_launch<64, MODE>(A, x, b, dinv, y, y2, gate, s, kind); break;
  }
}

// The V-cycle below expects the finest level's scratch `t` to hold the first
// l1-Jacobi iterate from zero, x0 = D^-1 b; the kernels that produce b also
// write x0 (restriction, the fracture-residual update, the input cast), so the
// smoother's residual needs one gather per nonzero.
template <typename T>
void start_smoother(DHier<T> &H, const T *b, const int *gate, hipStream_t s) {
  const int n = H.n();
  if (n == 0 || (H.lv.size() == 1 && H.dense)) return;
  timed_launch(kKcVcycleOther, s, 3.0 * sizeof(T) * n, [&] {
    hipLaunchKernelGGL(diag_scale_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, b,
                       dptr<const T>(H.lv[0].dinv), dptr<T>(H.lv[0].t), gate);
  });
}

template <typename T>
void coarse_solve(DHier<T> &H, const T *b, T *x, const int *gate, hipStream_t s) {
  DLevel<T> &L = H.lv.back();
  const int n = L.n;
  if (n == 0) return;
  if (H.dense) {
    const int blocks = (n + (kThreads / 64) - 1) / (kThreads / 64);
    timed_launch(kKcVcycleOther, s, 8.0 * n * n + 2.0 * sizeof(T) * n, [&] {
      hipLaunchKernelGGL(dense_gemv_kernel<T>, dim3(blocks), dim3(kThreads), 0, s, n, dptr<const double>(H.cinv),
                         b, x, gate);
    });
    return;
  }
  // four l1-Jacobi sweeps from zero: the first is x0 = D^-1 b, already in t
  T *pa = dptr<T>(H.tmp_pp), *pb = pa + n;
  const T *t = dptr<const T>(L.t);
  const T *dinv = dptr<const T>(L.dinv);
  const int kc = kKcVcycleOther;
  spmv<kSmooth>(L.A, t, b, dinv, pa, static_cast<T *>(nullptr), gate, s, kc);
  spmv<kSmooth>(L.A, static_cast<const T *>(pa), b, dinv, pb, static_cast<T *>(nullptr), gate, s, kc);
  spmv<kSmooth>(L.A, static_cast<const T *>(pb), b, dinv, x, static_cast<T *>(nullptr), gate, s, kc);
}

// One V-cycle from a zero initial guess: x = V(b), with lv[l].t = D^-1 b on entry.
template <typename T>
void vcycle(DHier<T> &H, size_t l, const T *b, T *x, const int *gate, hipStream_t s) {
  if (l + 1 == H.lv.size()) {
    coarse_solve(H, b, x, gate, s);
    return;
  }
  DLevel<T> &L = H.lv[l];
  DLevel<T> &C = H.lv[l + 1];
  T *t = dptr<T>(L.t);
  const T *dinv = dptr<const T>(L.dinv);
  const bool fine = H.is_omega && l == 0;
  const int ks = fine ? kKcFineSmooth : kKcVcycleOther;
  const int kr = fine ? kKcFineResid : kKcVcycleOther;
  const int ko = kKcVcycleOther;
  spmv<kResid>(L.A, static_cast<const T *>(t), b, dinv, dptr<T>(L.r), static_cast<T *>(nullptr), gate, s,
               kr);  // pre-smoothing x = t = D^-1 b done; r = b - A t
  spmv<kPlainScale>(L.R, dptr<const T>(L.r), static_cast<const T *>(nullptr), dptr<const T>(C.dinv), dptr<T>(C.b),
                    dptr<T>(C.t), gate, s, ko);  // b_c = R r, t_c = D_c^-1 b_c
  vcycle(H, l + 1, dptr<const T>(C.b), dptr<T>(C.x), gate, s);
  spmv<kAccum>(L.P, dptr<const T>(C.x), static_cast<const T *>(nullptr), static_cast<const T *>(nullptr), t,
               static_cast<T *>(nullptr), gate, s, ko);  // t += P x_c
  spmv<kSmooth>(L.A, static_cast<const T *>(t), b, dinv, x, static_cast<T *>(nullptr), gate, s, ks);  // post-smooth
}

// Q = `cycles` V-cycles as a stationary iteration from zero (lv[0].t = D^-1 r on entry).
template <typename T>
void apply_q(DHier<T> &H, int cycles, const T *r, T *z, const int *gate, hipStream_t s) {
  vcycle(H, 0, r, z, gate, s);
  const int n = H.n();
  for (int c = 1; c < cycles; ++c) {
    spmv<kResidScale>(H.lv[0].A, static_cast<const T *>(z), r, dptr<const T>(H.lv[0].dinv), dptr<T>(H.tmp_res),
                      dptr<T>(H.lv[0].t), gate, s, kKcVcycleOther);
    vcycle(H, 0, dptr<const T>(H.tmp_res), dptr<T>(H.tmp_dz), gate, s);
    hipLaunchKernelGGL(add_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, dptr<const T>(H.tmp_dz), z,
                       gate);
  }
}

// Algorithm 1: z = M_L r, with r and z laid out as [Omega; Gamma].  On entry
// Ho.lv[0].t = D^-1 r_O (see start_smoother).
template <typename T>
void apply_ml(Precond<T> &P, const T *r, T *z, const int *gate, hipStream_t s) {
  apply_q(P.Ho, P.vcycles, r, z, gate, s);  // z_O = Q_OO r_O
  if (P.n_g == 0) return;
  T *rg = dptr<T>(P.rg);
  spmv<kResidScale>(P.Ago, static_cast<const T *>(z), r + P.n_o, dptr<const T>(P.Hg.lv[0].dinv), rg,
                    dptr<T>(P.Hg.lv[0].t), gate, s, kKcVcycleOther);  // r_G - A_GO z_O (and D^-1 of it)
  apply_q(P.Hg, P.vcycles, static_cast<const T *>(rg), z + P.n_o, gate, s);  // z_G = Q_GG r_G
}

template <typename T>
std::unique_ptr<Precond<T>> upload_precond(const HostSystem &h, int vcycles, hipStream_t s) {
  auto p = std::make_unique<Precond<T>>();
  std::vector<std::vector<T>> keep;
  p->n_o = h.n_o;
  p->n_g = h.n_g;
  p->vcycles = vcycles;
  upload_hier(h.Ho, p->Ho, s, keep);
  p->Ho.is_omega = true;
  if (h.n_g > 0) {
    upload_hier(h.Hg, p->Hg, s, keep);
    upload_csr(h.Ago, p->Ago, s, keep);
    p->rg.alloc(static_cast<size_t>(h.n_g) * sizeof(T));
  }
  MDP_HIP(hipStreamSynchronize(s));  // host staging vectors die here
  return p;
}

int dcgs_blocks(int64_t n) { return static_cast<int>((n + kThreads * kDotU - 1) / (kThreads * kDotU)); }

template <typename TZ>
void update_x(int64_t n, int ncols, const TZ *Z, int64_t ld, const double *y, double *x, hipStream_t s) {
  timed_launch(kKcOther, s, (16.0 + sizeof(TZ) * ncols) * n, [&] {
    hipLaunchKernelGGL((update_x_kernel<TZ>), dim3(dcgs_blocks(n)), dim3(kThreads), 0, s, n, ncols, Z, ld, y, x);
  });
}

// ||v|| into ws.scalar (device) and returned to the host (synchronises s).
double norm_sync(Workspace &ws, int64_t n, const double *v, hipStream_t s) {
  hipLaunchKernelGGL(norm2_partial_kernel, dim3(kRedBlocks), dim3(kThreads), 0, s, n, v, dptr<double>(ws.npartial));
  hipLaunchKernelGGL(reduce_scalar_kernel, dim3(1), dim3(kThreads), 0, s, dptr<const double>(ws.npartial),
                     dptr<double>(ws.scalar), 1);
  MDP_HIP(hipMemcpyAsync(ws.host_scalar, ws.scalar.get(), sizeof(double), hipMemcpyDeviceToHost, s));
  MDP_HIP(hipStreamSynchronize(s));
  return *ws.host_scalar;
}

template <typename T>
int fgmres(Solver &S, Precond<T> &P, const double *b, double *x, hipStream_t s, mdp_stats *st) {
  Workspace &ws = S.ws;
  const int64_t n = S.n, ld = ws.ld;
  const int m = ws.m;
  const bool use_x0 = (S.opt.flags & MDP_USE_X0) != 0;
  double *V = dptr<double>(ws.V);
  T *Z = dptr<T>(ws.Z);
  double *w = dptr<double>(ws.w);
  GmresState *dst = dptr<GmresState>(ws.state);

  // caller order -> [Omega; Gamma]
  const double *bp = b;
  double *xp = x;
  if (!S.host.identity) {
    const int g = grid_for(n);
    hipLaunchKernelGGL(permute_kernel<true>, dim3(g), dim3(kThreads), 0, s, S.n, dptr<const int>(S.perm), b,
                       dptr<double>(ws.bp));
    bp = dptr<const double>(ws.bp);
    xp = dptr<double>(ws.xp);
    if (use_x0)
      hipLaunchKernelGGL(permute_kernel<true>, dim3(g), dim3(kThreads), 0, s, S.n, dptr<const int>(S.perm), x, xp);
  }
  const double bnorm = norm_sync(ws, n, bp, s);
  mdp_stats out{};
  if (!std::isfinite(bnorm)) {
    out.status = MDP_ENAN;
    if (st) *st = out;
    return MDP_ENAN;
  }
  if (!use_x0) MDP_HIP(hipMemsetAsync(xp, 0, n * sizeof(double), s));
  if (bnorm == 0.0) {
    if (use_x0) MDP_HIP(hipMemsetAsync(xp, 0, n * sizeof(double), s));
    if (!S.host.identity)
      hipLaunchKernelGGL(permute_kernel<false>, dim3(grid_for(n)), dim3(kThreads), 0, s, S.n,
                         dptr<const int>(S.perm), static_cast<const double *>(xp), x);
    MDP_HIP(hipStreamSynchronize(s));
    out.converged = 1;
    out.status = MDP_OK;
    if (st) *st = out;
    return MDP_OK;
  }
  const double tol_abs = S.opt.rtol * bnorm;
  double beta;
  if (use_x0) {
    spmv<kResid>(S.A, static_cast<const double *>(xp), bp, static_cast<const double *>(nullptr), V,
                 static_cast<double *>(nullptr), static_cast<const int *>(nullptr), s);
    beta = norm_sync(ws, n, V, s);
  } else {
    MDP_HIP(hipMemcpyAsync(V, bp, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    beta = bnorm;  // ws.scalar holds ||b|| = ||r_0||
  }

  int iters = 0, cycles = 0, code = MDP_OK;
  double est = beta;
  const int nblk = dcgs_blocks(n);
  const int *gate_apply = &dst->skip_apply;
  const int *gate_done = &dst->done;
  while (true) {
    if (!std::isfinite(beta)) {
      code = MDP_ENAN;
      break;
    }
    if (beta <= tol_abs || iters >= S.opt.max_iter) break;
    const int kmax = std::min(m, S.opt.max_iter - iters);
    // V[:, 0] holds the residual of the cycle start, unnormalised.
    hipLaunchKernelGGL(cycle_init_kernel, dim3(1), dim3(64), 0, s, dst, dptr<double>(ws.g), m);
    int last = -1;
    // Steps 0..kmax-1 apply the preconditioner; step kmax (if reached) only
    // finalises the last Hessenberg column.
    for (int j = 0; j <= kmax; ++j) {
      const KtBytes kt_before = ktimer_bytes();
      T *zj = Z + std::min(j, kmax - 1) * ld;
      const double *uj = V + j * ld;
      const T *pin;
      if constexpr (std::is_same<T, double>::value) {
        pin = uj;
        start_smoother(P.Ho, pin, gate_apply, s);
      } else {
        T *rin = dptr<T>(ws.rin);
        const int no = P.n_o;
        const bool need_t = !(P.Ho.lv.size() == 1 && P.Ho.dense);
        timed_launch(kKcOther, s, 12.0 * n + 8.0 * no, [&] {
          hipLaunchKernelGGL(cast_start_kernel, dim3(grid_for(n)), dim3(kThreads), 0, s, n, no, uj, rin,
                             dptr<const float>(P.Ho.lv[0].dinv), need_t ? dptr<float>(P.Ho.lv[0].t) : nullptr,
                             gate_apply);
        });
        pin = rin;
      }
      apply_ml(P, pin, zj, gate_apply, s);
      spmv<kPlain>(S.A, static_cast<const T *>(zj), static_cast<const double *>(nullptr),
                   static_cast<const double *>(nullptr), w, static_cast<double *>(nullptr), gate_apply, s,
                   kKcOuterSpmv);
      const int nv = 2 * j + 3;
      timed_launch(kKcArnoldiDot, s, 8.0 * n * (j + 2), [&] {
        hipLaunchKernelGGL(dcgs_reduce_kernel, dim3(nblk), dim3(kThreads), 0, s, n, j, static_cast<const double *>(V),
                           ld, static_cast<const double *>(w), dptr<double>(ws.partial), nblk, gate_done);
      });
      timed_launch(kKcOther, s, 8.0 * nv * nblk, [&] {
        hipLaunchKernelGGL(block_sums_kernel, dim3(nv), dim3(kThreads), 0, s, nv, dptr<const double>(ws.partial),
                           nblk, dptr<double>(ws.sums), gate_done);
      });
      timed_launch(kKcOther, s, 0.0, [&] {
        hipLaunchKernelGGL(dcgs_finalize_kernel, dim3(1), dim3(64), 0, s, dst, j, kmax, tol_abs,
                           dptr<const double>(ws.sums), dptr<double>(ws.hprev), dptr<DcgsCoef>(ws.coef),
                           dptr<double>(ws.Hr), m + 1, dptr<double>(ws.cs), dptr<double>(ws.sn),
                           dptr<double>(ws.g), dptr<double>(ws.hist));
      });
      timed_launch(kKcArnoldiAxpy, s, 8.0 * n * (j + 4), [&] {
        hipLaunchKernelGGL(dcgs_update_kernel, dim3(nblk), dim3(kThreads), 0, s, n, j, V, ld,
                           static_cast<const double *>(w), dptr<const DcgsCoef>(ws.coef), gate_done);
      });
      MDP_HIP(hipMemcpyAsync(&ws.host_state[j], dst, sizeof(GmresState), hipMemcpyDeviceToHost, s));
      MDP_HIP(hipEventRecord(ws.ev[j], s));
      last = j;
      if (j >= 1) {
        MDP_HIP(hipEventSynchronize(ws.ev[j - 1]));
        if (ws.host_state[j - 1].done) {
          ktimer_restore_bytes(kt_before);  // step j was queued after the cycle ended: a no-op
          break;
        }
      }
    }
    MDP_HIP(hipGetLastError());
    MDP_HIP(hipEventSynchronize(ws.ev[last]));
    const GmresState fs = ws.host_state[last];
    if (fs.nan) {
      code = MDP_ENAN;
      break;
    }
    const int k = fs.k;
    est = fs.est;
    iters += k;
    ++cycles;
    hipLaunchKernelGGL(backsolve_kernel, dim3(1), dim3(64), 0, s, static_cast<const GmresState *>(dst),
                       dptr<const double>(ws.Hr), m + 1, dptr<const double>(ws.g), dptr<double>(ws.y));
    update_x(n, k, static_cast<const T *>(Z), ld, dptr<const double>(ws.y), xp, s);
    spmv<kResid>(S.A, static_cast<const double *>(xp), bp, static_cast<const double *>(nullptr), V,
                 static_cast<double *>(nullptr), static_cast<const int *>(nullptr), s);
    beta = norm_sync(ws, n, V, s);
  }
  if (!S.host.identity)
    hipLaunchKernelGGL(permute_kernel<false>, dim3(grid_for(n)), dim3(kThreads), 0, s, S.n,
                       dptr<const int>(S.perm), static_cast<const double *>(xp), x);
  MDP_HIP(hipGetLastError());
  MDP_HIP(hipStreamSynchronize(s));
  out.iters = iters;
  out.restarts = std::max(cycles - 1, 0);
  out.rel_res_true = beta / bnorm;
  out.rel_res_est = est / bnorm;
  out.converged = (code == MDP_OK && beta <= tol_abs) ? 1 : 0;
  if (code == MDP_OK && !out.converged) code = MDP_NOT_CONVERGED;
  out.status = code;
  if (st) *st = out;
  return code;
}

}  // namespace

Workspace::~Workspace() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  if (host_state) (void)hipHostFree(host_state);
  if (host_scalar) (void)hipHostFree(host_scalar);
}

void Solver::upload(hipStream_t s) {
  n = host.n;
  n_o = host.n_o;
  n_g = host.n_g;
  std::vector<std::vector<double>> keep;
  upload_csr(host.A, A, s, keep);
  if (!host.identity) upload_vec(perm, host.perm, s);
  if (opt.precision == MDP_MIXED)
    pc32 = upload_precond<float>(host, opt.vcycles, s);
  else
    pc64 = upload_precond<double>(host, opt.vcycles, s);

  const size_t tsz = opt.precision == MDP_MIXED ? sizeof(float) : sizeof(double);
  ws.m = opt.restart;
  ws.ld = padded_ld(n);
  const size_t col8 = static_cast<size_t>(ws.ld) * sizeof(double);
  ws.V.alloc(col8 * (ws.m + 1));
  ws.Z.alloc(static_cast<size_t>(ws.ld) * tsz * ws.m);
  ws.w.alloc(col8);
  ws.rin.alloc(static_cast<size_t>(ws.ld) * tsz);
  if (!host.identity) {
    ws.bp.alloc(col8);
    ws.xp.alloc(col8);
  }
  const size_t mm = static_cast<size_t>(ws.m) + 1;
  for (DevMem *d : {&ws.cs, &ws.sn, &ws.g, &ws.y, &ws.hist, &ws.hprev}) d->alloc(mm * sizeof(double));
  ws.Hr.alloc(mm * ws.m * sizeof(double));
  ws.coef.alloc(sizeof(DcgsCoef));
  ws.sums.alloc((2 * mm + 3) * sizeof(double));
  ws.partial.alloc((2 * mm + 3) * static_cast<size_t>(dcgs_blocks(n)) * sizeof(double));
  ws.npartial.alloc(kRedBlocks * sizeof(double));
  ws.scalar.alloc(sizeof(double));
  ws.state.alloc(sizeof(GmresState));
  MDP_HIP(hipHostMalloc(reinterpret_cast<void **>(&ws.host_state), mm * sizeof(GmresState), hipHostMallocDefault));
  MDP_HIP(hipHostMalloc(reinterpret_cast<void **>(&ws.host_scalar), sizeof(double), hipHostMallocDefault));
  ws.ev.resize(mm);
  for (auto &e : ws.ev) MDP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  MDP_HIP(hipStreamSynchronize(s));
  on_device = true;
}

int Solver::solve(const double *b, double *x, hipStream_t s, mdp_stats *st) {
  const auto t0 = std::chrono::steady_clock::now();
  int rc = opt.precision == MDP_MIXED ? fgmres<float>(*this, *pc32, b, x, s, st)
                                      : fgmres<double>(*this, *pc64, b, x, s, st);
  const auto t1 = std::chrono::steady_clock::now();
  if (st) {
    st->solve_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    st->setup_ms = setup_ms;
  }
  return rc;
}

void Solver::apply(int op, const double *x, double *y, hipStream_t s) {
  const int64_t nn = n;
  switch (op) {
    case MDP_OP_A:
      spmv<kPlain>(A, x, static_cast<const double *>(nullptr), static_cast<const double *>(nullptr), y,
                   static_cast<double *>(nullptr), static_cast<const int *>(nullptr), s);
      break;
    case MDP_OP_ML:
    case MDP_OP_QOO:
    case MDP_OP_QGG: {
      const int64_t len = op == MDP_OP_ML ? nn : (op == MDP_OP_QOO ? n_o : n_g);
      if (len == 0) break;
      if (opt.precision == MDP_MIXED) {
        float *in = dptr<float>(ws.rin);
        float *out = dptr<float>(ws.Z);
        hipLaunchKernelGGL((scale_copy_kernel<double, float>), dim3(grid_for(len)), dim3(kThreads), 0, s, len, x,
                           static_cast<const double *>(nullptr), in, static_cast<const int *>(nullptr));
        auto &H = op == MDP_OP_QGG ? pc32->Hg : pc32->Ho;
        start_smoother(H, static_cast<const float *>(in), nullptr, s);
        if (op == MDP_OP_ML) apply_ml(*pc32, static_cast<const float *>(in), out, nullptr, s);
        else apply_q(H, pc32->vcycles, static_cast<const float *>(in), out, nullptr, s);
        hipLaunchKernelGGL((scale_copy_kernel<float, double>), dim3(grid_for(len)), dim3(kThreads), 0, s, len,
                           static_cast<const float *>(out), static_cast<const double *>(nullptr), y,
                           static_cast<const int *>(nullptr));
      } else {
        auto &H = op == MDP_OP_QGG ? pc64->Hg : pc64->Ho;
        start_smoother(H, x, nullptr, s);
        if (op == MDP_OP_ML) apply_ml(*pc64, x, y, nullptr, s);
        else apply_q(H, pc64->vcycles, x, y, nullptr, s);
      }
      break;
    }
    default:
      raise(MDP_EINVAL, "unknown operator");
  }
  MDP_HIP(hipGetLastError());
  MDP_HIP(hipStreamSynchronize(s));
}

}  // namespace mdp
