// HIP kernels for CDNA4 (gfx950): sparse products and l1-Jacobi smoothing of
// the AMG V-cycles, the dense coarsest solve, and the FP64 Arnoldi / Givens
// steps of flexible GMRES.
//
// Launch conventions: 256-thread workgroups (four 64-wide wavefronts).  Sparse
// kernels assign LPR lanes to a row (LPR a power of two <= 64), so one
// wavefront covers 64/LPR consecutive rows and its loads of column indices and
// values are contiguous.  Workgroups of the sparse kernels are renumbered so
// that each of the eight XCDs (which receive every eighth workgroup) walks one
// contiguous slice of rows: the gathered x entries then stay in that XCD's L2.
// Every kernel takes an optional device flag `gate`; when it is set the kernel
// returns at once (used to retire queued iterations after convergence).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "types.hpp"

namespace mdp {
namespace {  // each translation unit that launches kernels gets its own copy


template <typename A, typename B>
struct AccumT {
  using type = double;
};
template <>
struct AccumT<float, float> {
  using type = float;
};

__device__ __forceinline__ int xcd_block(int bid, int nblk) {
  const int xcd = bid % kXcds;
  const int local = bid / kXcds;
  const int per = nblk / kXcds, rem = nblk % kXcds;
  return xcd < rem ? xcd * (per + 1) + local : rem * (per + 1) + (xcd - rem) * per + local;
}

template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, W);
  return v;
}

enum SpmvMode : int {
  kPlain = 0,   // y = A x
  kResid = 1,   // y = b - A x
  kSmooth = 2,  // y = x + dinv .* (b - A x)          (one l1-Jacobi sweep, out of place)
  kPre0 = 3,    // y2 = dinv .* b ; y = b - A y2       (first sweep from zero, fused residual)
  kAccum = 4,   // y += A x                            (prolongation + correction)
};

template <int LPR, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void spmv_kernel(
    int nr, const int *__restrict__ ptr, const int *__restrict__ col, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk * (kThreads / LPR) + static_cast<int>(threadIdx.x) / LPR;
  const int lane = threadIdx.x % LPR;
  if (row >= nr) return;  // whole LPR groups leave together
  const int s = ptr[row], e = ptr[row + 1];
  Acc sum = 0;
  for (int p = s + lane; p < e; p += LPR) {
    const int c = col[p];
    Acc xv;
    if constexpr (MODE == kPre0)
      xv = static_cast<Acc>(b[c] * dinv[c]);
    else
      xv = static_cast<Acc>(x[c]);
    sum += static_cast<Acc>(val[p]) * xv;
  }
  sum = group_sum<LPR>(sum);
  if (lane == 0) {
    if constexpr (MODE == kPlain) {
      y[row] = static_cast<TY>(sum);
    } else if constexpr (MODE == kResid) {
      y[row] = static_cast<TY>(static_cast<Acc>(b[row]) - sum);
    } else if constexpr (MODE == kSmooth) {
      y[row] = static_cast<TY>(static_cast<Acc>(x[row]) +
                               static_cast<Acc>(dinv[row]) * (static_cast<Acc>(b[row]) - sum));
    } else if constexpr (MODE == kPre0) {
      y2[row] = b[row] * dinv[row];
      y[row] = static_cast<TY>(static_cast<Acc>(b[row]) - sum);
    } else {
      y[row] = static_cast<TY>(static_cast<Acc>(y[row]) + sum);
    }
  }
}

// Coarsest level: x = Ainv b with a dense FP64 inverse (row-major n x n); one
// wavefront per row, FP64 accumulation whatever the vector type.
template <typename T>
__global__ __launch_bounds__(kThreads) void dense_gemv_kernel(int n, const double *__restrict__ ainv,
                                                              const T *__restrict__ b,
                                                              T *__restrict__ x,
                                                              const int *__restrict__ gate) {
  if (gate && *gate) return;
  const int row = blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= n) return;
  const double *a = ainv + static_cast<size_t>(row) * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * static_cast<double>(b[j]);
  s = group_sum<64>(s);
  if (lane == 0) x[row] = static_cast<T>(s);
}

// out = in * (*scale) (scale may be null: 1), with a type conversion.
template <typename TI, typename TO>
__global__ __launch_bounds__(kThreads) void scale_copy_kernel(int64_t n, const TI *__restrict__ in,
                                                              const double *__restrict__ scale,
                                                              TO *__restrict__ out,
                                                              const int *__restrict__ gate) {
  if (gate && *gate) return;
  const double s = scale ? *scale : 1.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    out[i] = static_cast<TO>(static_cast<double>(in[i]) * s);
}

// x = b .* dinv
template <typename T>
__global__ __launch_bounds__(kThreads) void diag_scale_kernel(int n, const T *__restrict__ b,
                                                              const T *__restrict__ dinv,
                                                              T *__restrict__ x,
                                                              const int *__restrict__ gate) {
  if (gate && *gate) return;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads)
    x[i] = b[i] * dinv[i];
}

// y += x
template <typename T>
__global__ __launch_bounds__(kThreads) void add_kernel(int n, const T *__restrict__ x, T *__restrict__ y,
                                                       const int *__restrict__ gate) {
  if (gate && *gate) return;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) y[i] += x[i];
}

// out[perm[i]] = in[i]  (scatter)  or  out[i] = in[perm[i]]  (gather)
template <bool GATHER>
__global__ __launch_bounds__(kThreads) void permute_kernel(int n, const int *__restrict__ perm,
                                                           const double *__restrict__ in,
                                                           double *__restrict__ out) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) {
    if constexpr (GATHER)
      out[i] = in[perm[i]];
    else
      out[perm[i]] = in[i];
  }
}

// ---------------------------------------------------------------------------
// Block-level reduction helpers.  Deterministic: fixed tree inside the block.
template <typename T>
__device__ __forceinline__ T block_sum(T v, T *lds /* kThreads/64 entries */) {
  v = group_sum<64>(v);
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  T r = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < kThreads / 64; ++k) r += lds[k];
  }
  return r;  // valid in thread 0
}

// Contiguous element range of reduction block `blk` out of kRedBlocks.
__device__ __forceinline__ void red_range(int64_t n, int blk, int64_t &lo, int64_t &hi) {
  const int64_t chunk = (n + kRedBlocks - 1) / kRedBlocks;
  lo = blk * chunk;
  hi = lo + chunk < n ? lo + chunk : n;
}

// partial[i * kRedBlocks + blk] = sum_{e in range(blk)} V[e + i*ld] * w[e], i < ncols.
// NC: compile-time bound on ncols (8, 16, 32 or 64).
template <int NC>
__global__ __launch_bounds__(kThreads) void multi_dot_kernel(int64_t n, int ncols, const double *__restrict__ V,
                                                             int64_t ld, const double *__restrict__ w,
                                                             double *__restrict__ partial,
                                                             const int *__restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double lds[kThreads / 64];
  int64_t lo, hi;
  red_range(n, blockIdx.x, lo, hi);
  double acc[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) acc[i] = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
    const double we = w[e];
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (i < ncols) acc[i] += V[e + i * ld] * we;
  }
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    if (i >= ncols) break;
    const double s = block_sum(acc[i], lds);
    if (threadIdx.x == 0) partial[static_cast<int64_t>(i) * kRedBlocks + blockIdx.x] = s;
  }
}

// out[e] = w[e] - sum_i coef[i] * V[e + i*ld]  (out may alias w), and partial
// norms: partial[blk] = sum out[e]^2.
template <int NC>
__global__ __launch_bounds__(kThreads) void multi_axpy_kernel(int64_t n, int ncols, const double *__restrict__ V,
                                                              int64_t ld, const double *__restrict__ coef,
                                                              const double *w, double *out,
                                                              double *__restrict__ partial_norm,
                                                              const int *__restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double lds[kThreads / 64];
  __shared__ double c[NC];
  if (threadIdx.x < NC) c[threadIdx.x] = threadIdx.x < ncols ? coef[threadIdx.x] : 0.0;
  __syncthreads();
  int64_t lo, hi;
  red_range(n, blockIdx.x, lo, hi);
  double nrm = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) {
    double we = w[e];
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (i < ncols) we -= c[i] * V[e + i * ld];
    out[e] = we;
    nrm += we * we;
  }
  if (partial_norm) {
    const double s = block_sum(nrm, lds);
    if (threadIdx.x == 0) partial_norm[blockIdx.x] = s;
  }
}

// x[e] += sum_i y[i] * Z[e + i*ldz]  (Z in the preconditioner precision)
template <int NC, typename TZ>
__global__ __launch_bounds__(kThreads) void update_x_kernel(int64_t n, int ncols, const TZ *__restrict__ Z,
                                                            int64_t ldz, const double *__restrict__ y,
                                                            double *__restrict__ x) {
  __shared__ double c[NC];
  if (threadIdx.x < NC) c[threadIdx.x] = threadIdx.x < ncols ? y[threadIdx.x] : 0.0;
  __syncthreads();
  for (int64_t e = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; e < n;
       e += static_cast<int64_t>(gridDim.x) * kThreads) {
    double xe = x[e];
#pragma unroll
    for (int i = 0; i < NC; ++i)
      if (i < ncols) xe += c[i] * static_cast<double>(Z[e + i * ldz]);
    x[e] = xe;
  }
}

// partial[blk] = sum over the block's range of v[e]^2
__global__ __launch_bounds__(kThreads) void norm2_partial_kernel(int64_t n, const double *__restrict__ v,
                                                                  double *__restrict__ partial) {
  __shared__ double lds[kThreads / 64];
  int64_t lo, hi;
  red_range(n, blockIdx.x, lo, hi);
  double s = 0.0;
  for (int64_t e = lo + threadIdx.x; e < hi; e += kThreads) s += v[e] * v[e];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// One block per column i < ncols:
//   h[i] = scale[i] * sum_blk partial[i*kRedBlocks + blk];  coef[i] = h[i] * scale[i]
// (scale = per-column normalisation of the stored Krylov vectors).
__global__ __launch_bounds__(kThreads) void reduce_cols_kernel(int ncols, const double *__restrict__ partial,
                                                               const double *__restrict__ scale,
                                                               double *__restrict__ h,
                                                               double *__restrict__ coef,
                                                               const int *__restrict__ gate) {
  if (gate && *gate) return;
  __shared__ double lds[kThreads / 64];
  const int i = blockIdx.x;
  if (i >= ncols) return;
  double s = 0.0;
  for (int k = threadIdx.x; k < kRedBlocks; k += kThreads) s += partial[static_cast<int64_t>(i) * kRedBlocks + k];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) {
    const double hi = s * scale[i];
    h[i] = hi;
    coef[i] = hi * scale[i];
  }
}

// Sum of kRedBlocks partials into *out (single block), sqrt if requested.
__global__ __launch_bounds__(kThreads) void reduce_scalar_kernel(const double *__restrict__ partial,
                                                                 double *__restrict__ out, int take_sqrt) {
  __shared__ double lds[kThreads / 64];
  double s = 0.0;
  for (int k = threadIdx.x; k < kRedBlocks; k += kThreads) s += partial[k];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) *out = take_sqrt ? sqrt(s) : s;
}

// ---------------------------------------------------------------------------


// Start a cycle: beta = *rnorm, g = (beta, 0, ...), scale[0] = 1/beta.
__global__ void cycle_init_kernel(GmresState *st, const double *__restrict__ rnorm, double *__restrict__ g,
                                  double *__restrict__ scale, int m) {
  const double beta = *rnorm;
  for (int i = threadIdx.x; i <= m; i += blockDim.x) g[i] = 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    st->done = 0;
    st->k = 0;
    st->nan = !isfinite(beta);
    st->breakdown = 0;
    st->est = beta;
    st->beta = beta;
    g[0] = beta;
    scale[0] = 1.0 / beta;
  }
}

// Givens step for column j (single thread does the O(j) work):
//   H(:, j) = h1 + h2 (CGS2 coefficients), H(j+1, j) = ||w|| from partials.
// Applies the stored rotations, builds the new one, updates g, sets the
// residual estimate and the done flag (estimate <= tol_abs, breakdown, or j+1
// == kmax), and scale[j+1] = 1 / H(j+1, j).
__global__ __launch_bounds__(kThreads) void givens_kernel(GmresState *st, int j, int kmax, double tol_abs,
                                                          const double *__restrict__ h1,
                                                          const double *__restrict__ h2,
                                                          const double *__restrict__ norm_partial,
                                                          double *__restrict__ Hr /* (m+1) x m, col-major */,
                                                          int ldh, double *__restrict__ cs,
                                                          double *__restrict__ sn, double *__restrict__ g,
                                                          double *__restrict__ scale,
                                                          double *__restrict__ hist) {
  if (st->done) return;
  __shared__ double lds[kThreads / 64];
  double s = 0.0;
  for (int k = threadIdx.x; k < kRedBlocks; k += kThreads) s += norm_partial[k];
  s = block_sum(s, lds);
  if (threadIdx.x != 0) return;
  const double hn = sqrt(s);
  double *col = Hr + static_cast<int64_t>(j) * ldh;
  bool bad = !isfinite(hn);
  for (int i = 0; i <= j; ++i) {
    col[i] = h1[i] + h2[i];
    bad = bad || !isfinite(col[i]);
  }
  for (int i = 0; i < j; ++i) {
    const double t = cs[i] * col[i] + sn[i] * col[i + 1];
    col[i + 1] = -sn[i] * col[i] + cs[i] * col[i + 1];
    col[i] = t;
  }
  const double a = col[j], bb = hn;
  const double den = hypot(a, bb);
  const double c = a / den, sg = bb / den;
  cs[j] = c;
  sn[j] = sg;
  col[j] = den;
  col[j + 1] = 0.0;
  const double gj = g[j];
  g[j + 1] = -sg * gj;
  g[j] = c * gj;
  const double est = fabs(g[j + 1]);
  hist[j] = est;
  st->est = est;
  st->k = j + 1;
  const bool brk = (hn == 0.0);
  bad = bad || !isfinite(est);
  st->nan = bad;
  st->breakdown = brk;
  scale[j + 1] = brk ? 0.0 : 1.0 / hn;
  if (bad || brk || est <= tol_abs || j + 1 >= kmax) st->done = 1;
}

// Back substitution y = R(0:k,0:k)^{-1} g(0:k) for the k steps of the cycle.
__global__ void backsolve_kernel(const GmresState *st, const double *__restrict__ Hr, int ldh,
                                 const double *__restrict__ g, double *__restrict__ y) {
  if (threadIdx.x != 0) return;
  const int k = st->k;
  for (int i = k - 1; i >= 0; --i) {
    double s = g[i];
    for (int c = i + 1; c < k; ++c) s -= Hr[static_cast<int64_t>(c) * ldh + i] * y[c];
    y[i] = s / Hr[static_cast<int64_t>(i) * ldh + i];
  }
}

}  // namespace
}  // namespace mdp
