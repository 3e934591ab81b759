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
  kPlainScale = 5,  // y = A x ; y2 = dinv .* y         (restriction that also starts the coarse smoother)
  kResidScale = 6,  // y = b - A x ; y2 = dinv .* y     (residual that also starts the next smoother)
};

// Vector blocks of a sparse product: KB right-hand-side blocks share one
// matrix read; block r of x starts at r * xs, block r of b, dinv, y and y2
// at r * ys.  Batched solves skip, per block, the rows of pairs that have
// stopped applying the preconditioner (their output is no longer read): the
// pair of row i in block r is r * nsys + rpair[i] (rpair maps rows to
// systems; NULL means system 0).  Gating needs pst, and rpair or KB > 1.
struct Blocks {
  int64_t xs, ys;
  int nsys;
};

template <int KB>
__device__ __forceinline__ bool block_live(int row, int r, const int *__restrict__ rpair,
                                           const GmresState *__restrict__ pst, const Blocks &bk) {
  if (!pst || (!rpair && KB == 1)) return true;
  const int rp = rpair ? rpair[row] : 0;
  return !pst[r * bk.nsys + rp].skip_apply;
}

template <typename P>
__device__ __forceinline__ P *blk(P *p, int64_t off) {
  return p ? p + off : p;
}

// Per-row epilogue shared by the sparse kernels.
template <int MODE, typename Acc, typename TX, typename TY>
__device__ __forceinline__ void spmv_store(int row, Acc sum, const TX *__restrict__ x, const TY *__restrict__ b,
                                           const TY *__restrict__ dinv, TY *__restrict__ y, TY *__restrict__ y2) {
  if constexpr (MODE == kPlain) {
    y[row] = static_cast<TY>(sum);
  } else if constexpr (MODE == kResid) {
    y[row] = static_cast<TY>(static_cast<Acc>(b[row]) - sum);
  } else if constexpr (MODE == kSmooth) {
    y[row] = static_cast<TY>(static_cast<Acc>(x[row]) + static_cast<Acc>(dinv[row]) * (static_cast<Acc>(b[row]) - sum));
  } else if constexpr (MODE == kPre0) {
    y2[row] = b[row] * dinv[row];
    y[row] = static_cast<TY>(static_cast<Acc>(b[row]) - sum);
  } else if constexpr (MODE == kPlainScale) {
    const TY v = static_cast<TY>(sum);
    y[row] = v;
    y2[row] = v * dinv[row];
  } else if constexpr (MODE == kResidScale) {
    const TY v = static_cast<TY>(static_cast<Acc>(b[row]) - sum);
    y[row] = v;
    y2[row] = v * dinv[row];
  } else {
    y[row] = static_cast<TY>(static_cast<Acc>(y[row]) + sum);
  }
}

template <int MODE, typename Acc, typename TX, typename TY>
__device__ __forceinline__ Acc spmv_gather(int c, const TX *__restrict__ x, const TY *__restrict__ b,
                                           const TY *__restrict__ dinv) {
  if constexpr (MODE == kPre0)
    return static_cast<Acc>(b[c] * dinv[c]);
  else
    return static_cast<Acc>(x[c]);
}

// CSR-vector kernel for long rows: LPR lanes per row, each lane keeps BATCH
// entries in flight (indices and values loaded before the gathers).

template <int LPR, int BATCH, int KB, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void spmv_kernel(
    int nr, const int *__restrict__ ptr, const int *__restrict__ col, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate, const int *__restrict__ rpair,
    const GmresState *__restrict__ pst, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  const int blk_id = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk_id * (kThreads / LPR) + static_cast<int>(threadIdx.x) / LPR;
  const int lane = threadIdx.x % LPR;
  if (row >= nr) return;  // whole LPR groups leave together
  bool live[KB], any = false;
#pragma unroll
  for (int r = 0; r < KB; ++r) any |= (live[r] = block_live<KB>(row, r, rpair, pst, bk));
  if (!any) return;
  const int s = ptr[row], e = ptr[row + 1];
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  for (int p0 = s + lane; p0 < e; p0 += BATCH * LPR) {
    int c[BATCH];
    Acc v[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int p = p0 + k * LPR;
      // past the row end: value 0 and a column of this row (always in range)
      c[k] = p < e ? col[p] : col[s];
      v[k] = p < e ? static_cast<Acc>(val[p]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < BATCH; ++k)
          sum[r] += v[k] * spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys));
  }
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = group_sum<LPR>(sum[r]);
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
        spmv_store<MODE, Acc>(row, sum[r], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys), y + r * bk.ys,
                              blk(y2, r * bk.ys));
}

// CSR with one workgroup per row, for rows of hundreds to thousands of
// entries (the fused restrictions of the coarse levels): every thread keeps
// BATCH entries in flight, the wavefronts reduce their sums, and the first
// thread adds the kThreads / 64 wavefront sums in order.
template <int BATCH, int KB, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void spmv_row_block_kernel(
    int nr, const int *__restrict__ ptr, const int *__restrict__ col, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate, const int *__restrict__ rpair,
    const GmresState *__restrict__ pst, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  __shared__ Acc part[kThreads / 64][KB];
  const int row = xcd_block(blockIdx.x, gridDim.x);
  if (row >= nr) return;  // the whole workgroup leaves together
  bool live[KB], any = false;
#pragma unroll
  for (int r = 0; r < KB; ++r) any |= (live[r] = block_live<KB>(row, r, rpair, pst, bk));
  if (!any) return;
  const int t = static_cast<int>(threadIdx.x);
  const int s = ptr[row], e = ptr[row + 1];
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  for (int p0 = s + t; p0 < e; p0 += BATCH * kThreads) {
    int c[BATCH];
    Acc v[BATCH];
#pragma unroll
    for (int k = 0; k < BATCH; ++k) {
      const int p = p0 + k * kThreads;
      // past the row end: value 0 and a column of this row (always in range)
      c[k] = p < e ? col[p] : col[s];
      v[k] = p < e ? static_cast<Acc>(val[p]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < BATCH; ++k)
          sum[r] += v[k] * spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys));
  }
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = group_sum<64>(sum[r]);
  if (t % 64 == 0)
#pragma unroll
    for (int r = 0; r < KB; ++r) part[t / 64][r] = sum[r];
  __syncthreads();
  if (t != 0) return;
#pragma unroll
  for (int r = 0; r < KB; ++r) {
    if (!live[r]) continue;
    Acc tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) tot += part[w][r];
    spmv_store<MODE, Acc>(row, tot, x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys), y + r * bk.ys,
                          blk(y2, r * bk.ys));
  }
}

// Sliced ELL (slices of 64 rows = one wavefront, one thread per row): entry k
// of the row at lane L of slice s is stored at soff[s] + 64 k + L, so every
// load of indices and values is one contiguous 64-wide access.  Padding
// entries carry value 0 and a valid column.  The row loop is unrolled by
// kSellBatch so that many gathers are in flight per thread.
constexpr int kSellBatch = 8;

template <int KB, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void sell_kernel(
    int nr, int nslices, const int *__restrict__ soff, const int *__restrict__ col, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate, const int *__restrict__ rpair,
    const GmresState *__restrict__ pst, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  const int blk_id = xcd_block(blockIdx.x, gridDim.x);
  const int slice = blk_id * (kThreads / 64) + static_cast<int>(threadIdx.x) / 64;
  const int lane = threadIdx.x % 64;
  if (slice >= nslices) return;
  const int o0 = soff[slice], o1 = soff[slice + 1];
  const int row = slice * 64 + lane;
  if (row >= nr) return;
  bool live[KB], any = false;
#pragma unroll
  for (int r = 0; r < KB; ++r) any |= (live[r] = block_live<KB>(row, r, rpair, pst, bk));
  if (!any) return;
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  // kSellBatch entries per step, the last step predicated (past the slice
  // width: value 0 and this lane's first column), so that all index and
  // value loads of a short row are in flight together
  for (int o = o0 + lane; o < o1; o += kSellBatch * 64) {
    int c[kSellBatch];
    Acc v[kSellBatch];
#pragma unroll
    for (int k = 0; k < kSellBatch; ++k) {
      const int q = o + k * 64;
      c[k] = q < o1 ? col[q] : col[o];
      v[k] = q < o1 ? static_cast<Acc>(val[q]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < kSellBatch; ++k)
          sum[r] += v[k] * spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys));
  }
#pragma unroll
  for (int r = 0; r < KB; ++r)
    if (live[r])
      spmv_store<MODE, Acc>(row, sum[r], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys), y + r * bk.ys,
                            blk(y2, r * bk.ys));
}

// Diagonal storage for stencil matrices: entry (i, i + off[d]) is stored at
// val[d * nr + i] (zero where the matrix has no entry), with the offsets
// ascending, so each row is summed in column order as in the other formats.
// One thread per row; no column indices are read and the gathers of a
// wavefront are contiguous.
constexpr int kDiaBatch = 8;

template <int KB, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void dia_kernel(
    int nr, int nc, int ndiag, const int *__restrict__ off, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate, const int *__restrict__ rpair,
    const GmresState *__restrict__ pst, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  const int blk_id = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk_id * kThreads + static_cast<int>(threadIdx.x);
  if (row >= nr) return;
  bool live[KB], any = false;
#pragma unroll
  for (int r = 0; r < KB; ++r) any |= (live[r] = block_live<KB>(row, r, rpair, pst, bk));
  if (!any) return;
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  for (int d0 = 0; d0 < ndiag; d0 += kDiaBatch) {
    int c[kDiaBatch];
    bool in[kDiaBatch];
    Acc v[kDiaBatch];
#pragma unroll
    for (int k = 0; k < kDiaBatch; ++k) {
      const int d = d0 + k;
      c[k] = d < ndiag ? row + off[d] : row;
      in[k] = d < ndiag && c[k] >= 0 && c[k] < nc;
      v[k] = in[k] ? static_cast<Acc>(val[static_cast<int64_t>(d) * nr + row]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < kDiaBatch; ++k) {
          const Acc xv =
              in[k] ? spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys)) : Acc(0);
          sum[r] += v[k] * xv;
        }
  }
#pragma unroll
  for (int r = 0; r < KB; ++r)
    if (live[r])
      spmv_store<MODE, Acc>(row, sum[r], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys), y + r * bk.ys,
                            blk(y2, r * bk.ys));
}

// CSR with one thread per row, for short rows of uneven length (where slices
// would carry much padding): entries are loaded kScalarBatch at a time,
// predicated on the row length.
constexpr int kScalarBatch = 4;

template <int KB, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void csr_scalar_kernel(
    int nr, const int *__restrict__ ptr, const int *__restrict__ col, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate, const int *__restrict__ rpair,
    const GmresState *__restrict__ pst, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  const int blk_id = xcd_block(blockIdx.x, gridDim.x);
  const int row = blk_id * kThreads + static_cast<int>(threadIdx.x);
  if (row >= nr) return;
  bool live[KB], any = false;
#pragma unroll
  for (int r = 0; r < KB; ++r) any |= (live[r] = block_live<KB>(row, r, rpair, pst, bk));
  if (!any) return;
  const int s = ptr[row], e = ptr[row + 1];
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  for (int p0 = s; p0 < e; p0 += kScalarBatch) {
    int c[kScalarBatch];
    Acc v[kScalarBatch];
#pragma unroll
    for (int k = 0; k < kScalarBatch; ++k) {
      const int p = p0 + k;
      c[k] = p < e ? col[p] : col[s];
      v[k] = p < e ? static_cast<Acc>(val[p]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < kScalarBatch; ++k)
          sum[r] += v[k] * spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys));
  }
#pragma unroll
  for (int r = 0; r < KB; ++r)
    if (live[r])
      spmv_store<MODE, Acc>(row, sum[r], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys), y + r * bk.ys,
                            blk(y2, r * bk.ys));
}

// One colour of a multicolour Gauss-Seidel sweep (Section 4's smoother in a
// parallel order): the listed rows share a colour, so none of them reads
// another's update, and each is relaxed in place,
// x_i <- x_i + (b_i - sum_j a_ij x_j) / a_ii, LPR lanes per row, for KB
// right-hand-side blocks (strides as for the sparse products).
template <int LPR, int KB, typename TA, typename TY>
__global__ __launch_bounds__(kThreads) void gs_colour_kernel(int nrows, const int *__restrict__ rows,
                                                             const int *__restrict__ ptr, const int *__restrict__ col,
                                                             const TA *__restrict__ val, const TY *__restrict__ dg,
                                                             const TY *__restrict__ b, TY *x,
                                                             const int *__restrict__ gate, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TY>::type;
  const int k = static_cast<int>((static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x) / LPR);
  const int lane = threadIdx.x % LPR;
  if (k >= nrows) return;  // whole LPR groups leave together
  const int row = rows[k];
  const int s = ptr[row], e = ptr[row + 1];
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  for (int p = s + lane; p < e; p += LPR) {
    const int c = col[p];
    const Acc v = static_cast<Acc>(val[p]);
#pragma unroll
    for (int r = 0; r < KB; ++r) sum[r] += v * static_cast<Acc>(x[r * bk.xs + c]);
  }
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = group_sum<LPR>(sum[r]);
  if (lane == 0)
#pragma unroll
    for (int r = 0; r < KB; ++r) {
      const int64_t i = r * bk.ys + row;
      x[i] = static_cast<TY>(static_cast<Acc>(x[i]) + static_cast<Acc>(dg[i]) * (static_cast<Acc>(b[i]) - sum[r]));
    }
}

// Reads n 16-byte words and stores only if their sum equals the sentinel
// (never, for a buffer of zeros and a nonzero sentinel): it evicts the caches
// without leaving dirty lines behind.
__global__ __launch_bounds__(kThreads) void cache_flush_kernel(const double2 *__restrict__ p, int64_t n,
                                                               double sentinel, double *__restrict__ sink) {
  double acc = 0;
  const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const double2 v = p[i];
    acc += v.x + v.y;
  }
  if (acc == sentinel) sink[0] = acc;
}

// Row order of the diagonals-plus-remainder product.  Rows [split, nr) (the
// rows whose remainder gathers from far away) take the first blocks, padded to
// a multiple of kXcds blocks, so that they start first and spread over every
// XCD; rows [0, split) follow, each XCD taking a contiguous share of them.
// Rows past the end of their range get nr (the thread exits).
inline int hyb_blocks(int nr, int split) {
  const int tail = (nr - split + kThreads - 1) / kThreads;
  return (tail + kXcds - 1) / kXcds * kXcds + (split + kThreads - 1) / kThreads;
}

__device__ __forceinline__ int hyb_row(int nr, int split) {
  const int bid = static_cast<int>(blockIdx.x), t = static_cast<int>(threadIdx.x);
  const int tail = (nr - split + kThreads - 1) / kThreads;
  const int padded = (tail + kXcds - 1) / kXcds * kXcds;
  if (bid < padded) return bid < tail ? split + bid * kThreads + t : nr;
  const int row = xcd_block(bid - padded, static_cast<int>(gridDim.x) - padded) * kThreads + t;
  return row < split ? row : nr;
}

// Diagonals plus a CSR remainder, one thread per row: for stencil matrices
// with a few irregular couplings (the system matrix: the host's stencil on
// the diagonals; host-fracture and fracture-fracture couplings in the
// remainder).  Entry (i, i + doff[d]) of the diagonals is at dval[d * nr + i]
// (zero where absent, or past the columns); the remainder's row i holds the
// other entries of row i.  Diagonal terms are summed first, in offset order,
// then the remainder's in row order.
template <int KB, int MODE, typename TA, typename TX, typename TY>
__global__ __launch_bounds__(kThreads) void hyb_kernel(
    int nr, int nc, int split, int ndiag, const int *__restrict__ doff, const TA *__restrict__ dval,
    const int *__restrict__ ptr, const int *__restrict__ col, const TA *__restrict__ val,
    const TX *__restrict__ x, const TY *__restrict__ b, const TY *__restrict__ dinv,
    TY *__restrict__ y, TY *__restrict__ y2, const int *__restrict__ gate, const int *__restrict__ rpair,
    const GmresState *__restrict__ pst, Blocks bk) {
  if (gate && *gate) return;
  using Acc = typename AccumT<TA, TX>::type;
  const int row = hyb_row(nr, split);
  if (row >= nr) return;
  bool live[KB], any = false;
#pragma unroll
  for (int r = 0; r < KB; ++r) any |= (live[r] = block_live<KB>(row, r, rpair, pst, bk));
  if (!any) return;
  // the remainder's bounds and first entries are loaded before the diagonals
  // so that their latency overlaps the diagonal loads
  const int s = ptr[row], e = ptr[row + 1];
  int c0[kScalarBatch];
  Acc v0[kScalarBatch];
#pragma unroll
  for (int k = 0; k < kScalarBatch; ++k) {
    c0[k] = s + k < e ? col[s + k] : 0;
    v0[k] = s + k < e ? static_cast<Acc>(val[s + k]) : Acc(0);
  }
  Acc sum[KB];
#pragma unroll
  for (int r = 0; r < KB; ++r) sum[r] = 0;
  for (int d0 = 0; d0 < ndiag; d0 += kDiaBatch) {
    int c[kDiaBatch];
    bool in[kDiaBatch];
    Acc v[kDiaBatch];
#pragma unroll
    for (int k = 0; k < kDiaBatch; ++k) {
      const int d = d0 + k;
      c[k] = d < ndiag ? row + doff[d] : row;
      in[k] = d < ndiag && c[k] >= 0 && c[k] < nc;
      v[k] = in[k] ? static_cast<Acc>(dval[static_cast<int64_t>(d) * nr + row]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < kDiaBatch; ++k) {
          const Acc xv =
              in[k] ? spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys)) : Acc(0);
          sum[r] += v[k] * xv;
        }
  }
#pragma unroll
  for (int r = 0; r < KB; ++r)
    if (live[r])
#pragma unroll
      for (int k = 0; k < kScalarBatch; ++k)
        if (s + k < e)
          sum[r] += v0[k] * spmv_gather<MODE, Acc>(c0[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys));
  for (int p0 = s + kScalarBatch; p0 < e; p0 += kScalarBatch) {
    int c[kScalarBatch];
    Acc v[kScalarBatch];
#pragma unroll
    for (int k = 0; k < kScalarBatch; ++k) {
      const int p = p0 + k;
      c[k] = p < e ? col[p] : col[s];
      v[k] = p < e ? static_cast<Acc>(val[p]) : Acc(0);
    }
#pragma unroll
    for (int r = 0; r < KB; ++r)
      if (live[r])
#pragma unroll
        for (int k = 0; k < kScalarBatch; ++k)
          sum[r] += v[k] * spmv_gather<MODE, Acc>(c[k], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys));
  }
#pragma unroll
  for (int r = 0; r < KB; ++r)
    if (live[r])
      spmv_store<MODE, Acc>(row, sum[r], x + r * bk.xs, blk(b, r * bk.ys), blk(dinv, r * bk.ys), y + r * bk.ys,
                            blk(y2, r * bk.ys));
}

// Coarsest levels (dense FP64 inverses, row-major): x = Ainv_d b on each
// descriptor's rows; grid (ceil(max n / 4), ndesc), one wavefront per row,
// FP64 accumulation whatever the vector type.
template <typename T>
__global__ __launch_bounds__(kThreads) void dense_gemv_batched_kernel(const DenseDesc *__restrict__ desc,
                                                                      const double *__restrict__ ainv,
                                                                      const T *__restrict__ b, T *__restrict__ x,
                                                                      const int *__restrict__ gate) {
  if (gate && *gate) return;
  const DenseDesc d = desc[blockIdx.y];
  const int row = blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
  const int lane = threadIdx.x % 64;
  if (row >= d.n) return;
  const double *a = ainv + d.inv_off + static_cast<int64_t>(row) * d.n;
  const T *bb = b + d.row;
  // four partial sums, so that four loads per lane are in flight (few rows
  // per system: the wavefronts alone cannot hide the latency)
  double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
  int j = lane;
  for (; j + 192 < d.n; j += 256) {
    s0 += a[j] * static_cast<double>(bb[j]);
    s1 += a[j + 64] * static_cast<double>(bb[j + 64]);
    s2 += a[j + 128] * static_cast<double>(bb[j + 128]);
    s3 += a[j + 192] * static_cast<double>(bb[j + 192]);
  }
  for (; j < d.n; j += 64) s0 += a[j] * static_cast<double>(bb[j]);
  double s = (s0 + s1) + (s2 + s3);
  s = group_sum<64>(s);
  if (lane == 0) x[d.row + row] = static_cast<T>(s);
}

// Batched gather / scatter between the callers' vectors (one device pointer
// per pair, caller order) and the global layout.
__global__ __launch_bounds__(kThreads) void gather_pairs_kernel(int64_t n, const int *__restrict__ gpair,
                                                                const int *__restrict__ gidx,
                                                                const double *const *__restrict__ src,
                                                                double *__restrict__ out) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    out[i] = src[gpair[i]][gidx[i]];
}
__global__ __launch_bounds__(kThreads) void scatter_pairs_kernel(int64_t n, const int *__restrict__ gpair,
                                                                 const int *__restrict__ gidx,
                                                                 const double *__restrict__ in,
                                                                 double *const *__restrict__ dst,
                                                                 const int *__restrict__ active) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const int p = gpair[i];
    if (!active || active[p]) dst[p][gidx[i]] = in[i];
  }
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

// First preconditioner input of a cycle, one tile per workgroup: rin =
// (float)(u * scale[pair]) over the tile (the cycle's unnormalised residual
// brought to unit norm before the FP32 cast, so that no entry leaves FP32's
// range; FGMRES is unchanged by the scale of a preconditioned direction,
// since A z_j is formed from the stored z_j); t[i] = rin[i] * dinv[i] on the
// first no entries (the host block's first smoother iterate), when t is given.
__global__ __launch_bounds__(kThreads) void cast_start_kernel(const Tile *__restrict__ tiles, int64_t no,
                                                              const double *__restrict__ u,
                                                              const double *__restrict__ scale,
                                                              float *__restrict__ rin,
                                                              const float *__restrict__ dinv,
                                                              float *__restrict__ t,
                                                              const int *__restrict__ gate) {
  if (gate && *gate) return;
  const Tile tl = tiles[blockIdx.x];
  const double sc = scale[tl.pair];
  for (int k = threadIdx.x; k < tl.len; k += kThreads) {
    const int64_t i = tl.start + k;
    const float v = static_cast<float>(u[i] * sc);
    rin[i] = v;
    if (t && i < no) t[i] = v * dinv[i];
  }
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
// y[0..n) = 0 (a kernel rather than a memset node, so that captured graphs
// replay correctly).
template <typename T>
__global__ __launch_bounds__(kThreads) void zero_kernel(int n, T *__restrict__ y, const int *__restrict__ gate) {
  if (gate && *gate) return;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) y[i] = T(0);
}

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

// ---------------------------------------------------------------------------
// Arnoldi with classical Gram-Schmidt and delayed reorthogonalisation.
//
// At step j the basis V[:, 0..j-1] = q_0..q_{j-1} is final, V[:, j] = u_j is the
// provisional vector (orthogonalised once), and w = A z_j with z_j = M u_j.
// One fused pass computes a = Q^T u_j, b = Q^T w, alpha = u.u, beta = u.w,
// gamma = w.w; a small kernel then finalises column j-1 (u_j re-orthogonalised
// with a) and forms column j; one update pass writes q_j and u_{j+1}.

// Sum 8 values over the 64 lanes of a wavefront by recursive halving: after
// the call, every lane holds in v[0] the wave total of value index
// 4*bit5(L) + 2*bit4(L) + bit3(L) (see wave_reduce8_index).  10 shuffles
// instead of 48.
__device__ __forceinline__ void wave_reduce8(double v[8]) {
  const int lane = threadIdx.x % 64;
  {
    const bool hi = lane & 32;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const double send = hi ? v[k] : v[k + 4];
      const double keep = hi ? v[k + 4] : v[k];
      v[k] = keep + __shfl_xor(send, 32, 64);
    }
  }
  {
    const bool hi = lane & 16;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const double send = hi ? v[k] : v[k + 2];
      const double keep = hi ? v[k + 2] : v[k];
      v[k] = keep + __shfl_xor(send, 16, 64);
    }
  }
  {
    const bool hi = lane & 8;
    const double send = hi ? v[0] : v[1];
    const double keep = hi ? v[1] : v[0];
    v[0] = keep + __shfl_xor(send, 8, 64);
  }
  v[0] += __shfl_xor(v[0], 4, 64);
  v[0] += __shfl_xor(v[0], 2, 64);
  v[0] += __shfl_xor(v[0], 1, 64);
}

__device__ __forceinline__ int wave_reduce8_index(int lane) {
  return ((lane >> 5) & 1) * 4 + ((lane >> 4) & 1) * 2 + ((lane >> 3) & 1);
}

// Per-tile partial sums, part[v * ntiles + tile], of the 2*nq + 3 values
// [a_0..a_{nq-1}, b_0..b_{nq-1}, alpha, beta, gamma] of the tile's pair.
__global__ __launch_bounds__(kThreads) void dcgs_reduce_kernel(const Tile *__restrict__ tiles, int ntiles, int nq,
                                                               const double *__restrict__ V, int64_t ld,
                                                               const double *__restrict__ w,
                                                               double *__restrict__ part,
                                                               const GmresState *__restrict__ st) {
  const Tile tl = tiles[blockIdx.x];
  if (st[tl.pair].done) return;
  __shared__ double lds[kThreads / 64][2 * kMaxCols + 8];
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const int64_t base = tl.start + threadIdx.x;
  const int lim = tl.len - static_cast<int>(threadIdx.x);
  const double *u = V + static_cast<int64_t>(nq) * ld;
  double uu[kDotU], ww[kDotU];
#pragma unroll
  for (int k = 0; k < kDotU; ++k) {
    const bool in = k * kThreads < lim;
    uu[k] = in ? u[base + k * kThreads] : 0.0;
    ww[k] = in ? w[base + k * kThreads] : 0.0;
  }
  const int slot = wave_reduce8_index(lane);
  for (int c0 = 0; c0 < nq; c0 += 4) {
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      if (c0 + c < nq) {
        const double *q = V + static_cast<int64_t>(c0 + c) * ld;
#pragma unroll
        for (int k = 0; k < kDotU; ++k) {
          const double qe = k * kThreads < lim ? q[base + k * kThreads] : 0.0;
          acc[c] += qe * uu[k];
          acc[4 + c] += qe * ww[k];
        }
      }
    }
    wave_reduce8(acc);
    if ((lane & 7) == 0) {
      const int c = slot & 3;
      const int v = slot < 4 ? c0 + c : nq + c0 + c;
      if (c0 + c < nq) lds[wave][v] = acc[0];
    }
  }
  {
    double acc[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) acc[c] = 0.0;
#pragma unroll
    for (int k = 0; k < kDotU; ++k) {
      acc[0] += uu[k] * uu[k];
      acc[1] += uu[k] * ww[k];
      acc[2] += ww[k] * ww[k];
    }
    wave_reduce8(acc);
    if ((lane & 7) == 0 && slot < 3) lds[wave][2 * nq + slot] = acc[0];
  }
  __syncthreads();
  const int nv = 2 * nq + 3;
  for (int v = threadIdx.x; v < nv; v += kThreads) {
    double s = 0.0;
#pragma unroll
    for (int wv = 0; wv < kThreads / 64; ++wv) s += lds[wv][v];
    part[static_cast<int64_t>(v) * ntiles + blockIdx.x] = s;
  }
}

// sums[p * sstride + v] = sum over the tiles of pair p of part[v * ntiles + t];
// grid (nv, npairs).
__global__ __launch_bounds__(kThreads) void pair_sums_kernel(int nv, const double *__restrict__ part, int ntiles,
                                                             const int *__restrict__ tile_off,
                                                             double *__restrict__ sums, int sstride,
                                                             const GmresState *__restrict__ st) {
  __shared__ double lds[kThreads / 64];
  const int v = blockIdx.x, p = blockIdx.y;
  if (v >= nv || st[p].done) return;
  double s = 0.0;
  for (int t = tile_off[p] + threadIdx.x; t < tile_off[p + 1]; t += kThreads) s += part[static_cast<int64_t>(v) * ntiles + t];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) sums[static_cast<int64_t>(p) * sstride + v] = s;
}

// part[t] = sum over tile t of v[e]^2, for every tile (no gating).
__global__ __launch_bounds__(kThreads) void tile_norm2_kernel(const Tile *__restrict__ tiles,
                                                              const double *__restrict__ v,
                                                              double *__restrict__ part) {
  __shared__ double lds[kThreads / 64];
  const Tile tl = tiles[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < tl.len; i += kThreads) {
    const double x = v[tl.start + i];
    s += x * x;
  }
  s = block_sum(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// out[p] = sqrt(sum of the pair's tile partials); one block per pair.
__global__ __launch_bounds__(kThreads) void pair_norm_kernel(const double *__restrict__ part,
                                                             const int *__restrict__ tile_off,
                                                             double *__restrict__ out) {
  __shared__ double lds[kThreads / 64];
  const int p = blockIdx.x;
  double s = 0.0;
  for (int t = tile_off[p] + threadIdx.x; t < tile_off[p + 1]; t += kThreads) s += part[t];
  s = block_sum(s, lds);
  if (threadIdx.x == 0) out[p] = sqrt(s);
}

// Givens rotation that zeroes b in (a, b).
__device__ __forceinline__ void givens(double a, double b, double &c, double &s, double &r) {
  r = hypot(a, b);
  c = a / r;
  s = b / r;
}

// Mark pair state `s` as no longer applying the preconditioner / as finished,
// maintaining the batch-wide counters.
__device__ __forceinline__ void pair_stop_apply(GmresState *s, BatchCtl *ctl) {
  if (!s->skip_apply) {
    s->skip_apply = 1;
    if (atomicSub(&ctl->napply_left, 1) == 1) ctl->skip_all_apply = 1;
  }
}
__device__ __forceinline__ void pair_finish(GmresState *s, BatchCtl *ctl, int npairs) {
  pair_stop_apply(s, ctl);
  s->done = 1;
  if (atomicAdd(&ctl->ndone, 1) == npairs - 1) ctl->all_done = 1;
}

// Step j of the cycle for pair blockIdx.x (one wavefront):
//  * j > 0: re-orthogonalise u_j against q_0..q_{j-1} (coefficients a) and
//    finalise Hessenberg column j-1 = hprev + nu a, with subdiagonal nu r;
//    apply the stored rotations, form rotation j-1, update g; the estimate
//    |g_j| is final for basis size j.  Stop if it meets the tolerance or if
//    the previous step announced that this step only finalises.
//  * form column j from b, beta (its provisional subdiagonal from gamma),
//    estimate the residual of basis size j+1 with a trial rotation, and
//    announce the last step when that estimate meets the tolerance, when
//    j+1 == kmax, or on (near) breakdown.  Write the update-pass coefficients.
// Per-pair arrays are laid out with the strides ldh*m (Hr), ldv (vectors of
// length m+1) and sstride (sums).
__global__ __launch_bounds__(64) void dcgs_finalize_kernel(GmresState *__restrict__ st_all, BatchCtl *ctl, int npairs,
                                                           int j, const int *__restrict__ kmaxp,
                                                           const double *__restrict__ tolp,
                                                           const double *__restrict__ sums_all, int sstride,
                                                           double *__restrict__ hprev_all, DcgsCoef *cf_all,
                                                           double *__restrict__ Hr_all, int ldh, int m,
                                                           double *__restrict__ cs_all, double *__restrict__ sn_all,
                                                           double *__restrict__ g_all, double *__restrict__ hist_all,
                                                           int ldv) {
  // One wavefront per pair: the O(j) vector work (loads, dot products,
  // column updates, stores) is spread over the 64 lanes; lane 0 runs the two
  // rotation chains and the scalar decisions.
  const int p = blockIdx.x;
  GmresState *st = st_all + p;
  if (st->done) return;
  const double *sums = sums_all + static_cast<int64_t>(p) * sstride;
  double *hprev = hprev_all + static_cast<int64_t>(p) * ldv;
  double *cs = cs_all + static_cast<int64_t>(p) * ldv;
  double *sn = sn_all + static_cast<int64_t>(p) * ldv;
  double *g = g_all + static_cast<int64_t>(p) * ldv;
  double *hist = hist_all + static_cast<int64_t>(p) * ldv;
  double *Hr = Hr_all + static_cast<int64_t>(p) * ldh * m;
  DcgsCoef *cf = cf_all + p;
  const int kmax = kmaxp[p];
  const double tol_abs = tolp[p];
  __shared__ double a[kMaxCols + 1], b[kMaxCols + 1], col[kMaxCols + 2], sc[kMaxCols + 1], ss[kMaxCols + 1];
  __shared__ int stop;
  const int t = threadIdx.x;
  double paa = 0.0, pab = 0.0, pbb = 0.0;
  for (int i = t; i < j; i += 64) {
    const double ai = sums[i], bi = sums[j + i];
    a[i] = ai;
    b[i] = bi;
    sc[i] = cs[i];
    ss[i] = sn[i];
    col[i] = hprev[i];
    paa += ai * ai;
    pab += ai * bi;
    pbb += bi * bi;
  }
  const double alpha = sums[2 * j], beta = sums[2 * j + 1], gamma = sums[2 * j + 2];
  const double saa = group_sum<64>(paa), sab = group_sum<64>(pab), sbb = group_sum<64>(pbb);
  bool bad = !isfinite(alpha) || !isfinite(beta) || !isfinite(gamma);
  const double r2 = alpha - saa;
  const double r = sqrt(r2 > 1e-30 * alpha ? r2 : 1e-30 * alpha);
  if (t == 0) stop = 0;
  if (j == 0) {
    if (t == 0) g[0] = r;  // the cycle's first vector is the unnormalised residual
  } else {
    const double nu = st->nu;
    for (int i = t; i < j; i += 64) col[i] += nu * a[i];
    if (t == 0) col[j] = nu * r;
    __syncthreads();
    if (t == 0) {
      // apply the stored rotations; the rotated entry carried to the next
      // rotation stays in a register
      double cur = col[0];
      for (int i = 0; i + 1 < j; ++i) {
        const double nxt = col[i + 1];
        const double tt = sc[i] * cur + ss[i] * nxt;
        cur = -ss[i] * cur + sc[i] * nxt;
        col[i] = tt;
      }
      col[j - 1] = cur;
      double c, s, rr;
      givens(col[j - 1], col[j], c, s, rr);
      cs[j - 1] = c;
      sn[j - 1] = s;
      col[j - 1] = rr;
      col[j] = 0.0;
      const double gj = g[j - 1];
      g[j] = -s * gj;
      g[j - 1] = c * gj;
      const double est = fabs(g[j]);
      hist[j - 1] = est;
      st->k = j;
      st->est = est;
      const bool bad1 = bad || !isfinite(est);
      if (bad1 || st->finishing || est <= tol_abs) {
        st->nan = bad1;
        pair_finish(st, ctl, npairs);
        stop = 1;
      }
      sc[j - 1] = c;  // the rotations now include the one just formed
      ss[j - 1] = s;
    }
    __syncthreads();
    for (int i = t; i <= j; i += 64) Hr[static_cast<int64_t>(j - 1) * ldh + i] = col[i];
    if (stop) return;
    __syncthreads();  // col is rewritten below
  }
  // provisional column j
  const double hj = (beta - sab) / r;
  const double sh = sbb + hj * hj;
  for (int i = t; i < j; i += 64) col[i] = b[i];
  if (t == 0) col[j] = hj;
  const double nu2 = gamma - sh;
  const bool brk = !(nu2 > 1e-24 * gamma);
  const double nu = sqrt(brk ? fmax(1e-24 * gamma, 1e-300) : nu2);
  __syncthreads();
  for (int i = t; i <= j; i += 64) hprev[i] = col[i];
  for (int i = t; i < j; i += 64) {
    cf->a[i] = a[i];
    cf->b[i] = b[i];
  }
  if (t != 0) return;
  // only the last entry of the rotated provisional column is needed: carry it
  double cur = col[0];
  for (int i = 0; i < j; ++i) cur = -ss[i] * cur + sc[i] * col[i + 1];
  double c, s, rr;
  givens(cur, nu, c, s, rr);
  const double est_next = fabs(s * g[j]);
  bad = bad || !isfinite(hj) || !isfinite(nu) || !(r > 0.0);
  cf->inv_r = 1.0 / r;
  cf->hj = hj;
  cf->inv_nu = 1.0 / nu;
  st->nu = nu;
  st->nan = bad;
  if (bad) {
    pair_finish(st, ctl, npairs);
    return;
  }
  if (brk || est_next <= tol_abs || j + 1 >= kmax) {
    st->finishing = 1;
    pair_stop_apply(st, ctl);
  }
}

// q_j = (u_j - sum_i a_i q_i) * inv_r ;  u_{j+1} = (w - sum_i b_i q_i - hj q_j) * inv_nu
// on one tile of one pair.
__global__ __launch_bounds__(kThreads) void dcgs_update_kernel(const Tile *__restrict__ tiles, int nq,
                                                               double *__restrict__ V, int64_t ld,
                                                               const double *__restrict__ w,
                                                               const DcgsCoef *__restrict__ cf_all,
                                                               const GmresState *__restrict__ st,
                                                               NextInput nin) {
  if (nin.host_ctl && blockIdx.x == 0 && threadIdx.x == 0) {
    *nin.host_ctl = *nin.ctl;  // final for this step: the finalise kernel ran before
    __threadfence_system();
  }
  const Tile tl = tiles[blockIdx.x];
  if (st[tl.pair].done) return;
  const DcgsCoef *cf = cf_all + tl.pair;
  const int64_t base = tl.start + threadIdx.x;
  const int lim = tl.len - static_cast<int>(threadIdx.x);
  double *u = V + static_cast<int64_t>(nq) * ld;
  double *un = u + ld;
  double uu[kDotU], ww[kDotU];
#pragma unroll
  for (int k = 0; k < kDotU; ++k) {
    const bool in = k * kThreads < lim;
    uu[k] = in ? u[base + k * kThreads] : 0.0;
    ww[k] = in ? w[base + k * kThreads] : 0.0;
  }
  // newest columns first: the reduction pass has just read them, so they are
  // the ones still in the Infinity Cache
  int i = nq;
  for (; i >= 4; i -= 4) {
    double ca[4], cb[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ca[c] = cf->a[i - 1 - c];
      cb[c] = cf->b[i - 1 - c];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const double *q = V + static_cast<int64_t>(i - 1 - c) * ld;
#pragma unroll
      for (int k = 0; k < kDotU; ++k) {
        const double qe = k * kThreads < lim ? q[base + k * kThreads] : 0.0;
        uu[k] -= ca[c] * qe;
        ww[k] -= cb[c] * qe;
      }
    }
  }
  for (; i > 0; --i) {
    const double ca = cf->a[i - 1], cb = cf->b[i - 1];
    const double *q = V + static_cast<int64_t>(i - 1) * ld;
#pragma unroll
    for (int k = 0; k < kDotU; ++k) {
      const double qe = k * kThreads < lim ? q[base + k * kThreads] : 0.0;
      uu[k] -= ca * qe;
      ww[k] -= cb * qe;
    }
  }
  const double inv_r = cf->inv_r, hj = cf->hj, inv_nu = cf->inv_nu;
#pragma unroll
  for (int k = 0; k < kDotU; ++k) {
    if (k * kThreads < lim) {
      const int64_t e = base + k * kThreads;
      const double qj = uu[k] * inv_r;
      u[e] = qj;
      const double next = (ww[k] - hj * qj) * inv_nu;
      un[e] = next;
      if (nin.rin) {  // FP32 copy; u_{j+1} is already scaled to unit norm
        const float v = static_cast<float>(next);
        nin.rin[e] = v;
        if (nin.t32 && e < nin.n_o) nin.t32[e] = v * nin.dinv32[e];
      } else if (nin.t64 && e < nin.n_o) {  // same arithmetic as diag_scale_kernel
        nin.t64[e] = next * nin.dinv64[e];
      }
    }
  }
}

// x[e] += sum_{i < k} y[i] * Z[e + i*ldz] on one tile, k and y of the tile's pair.
template <typename TZ>
__global__ __launch_bounds__(kThreads) void update_x_kernel(const Tile *__restrict__ tiles, const TZ *__restrict__ Z,
                                                            int64_t ldz, const double *__restrict__ y_all, int ldv,
                                                            const GmresState *__restrict__ st,
                                                            const int *__restrict__ active,
                                                            double *__restrict__ x) {
  const Tile tl = tiles[blockIdx.x];
  if (!active[tl.pair]) return;
  const int ncols = st[tl.pair].k;
  const double *y = y_all + static_cast<int64_t>(tl.pair) * ldv;
  const int64_t base = tl.start + threadIdx.x;
  const int lim = tl.len - static_cast<int>(threadIdx.x);
  double xx[kDotU];
#pragma unroll
  for (int k = 0; k < kDotU; ++k) xx[k] = k * kThreads < lim ? x[base + k * kThreads] : 0.0;
  for (int i = 0; i < ncols; ++i) {
    const double yi = y[i];
    const TZ *z = Z + static_cast<int64_t>(i) * ldz;
#pragma unroll
    for (int k = 0; k < kDotU; ++k)
      if (k * kThreads < lim) xx[k] += yi * static_cast<double>(z[base + k * kThreads]);
  }
#pragma unroll
  for (int k = 0; k < kDotU; ++k)
    if (k * kThreads < lim) x[base + k * kThreads] = xx[k];
}

// Start a cycle: per pair, clear the state and g (done = not active); pair 0's
// block also resets the batch control words.
__global__ __launch_bounds__(64) void cycle_init_kernel(GmresState *__restrict__ st, BatchCtl *ctl, int npairs,
                                                        int nactive, const int *__restrict__ active,
                                                        double *__restrict__ g_all, int ldv) {
  const int p = blockIdx.x;
  double *g = g_all + static_cast<int64_t>(p) * ldv;
  for (int i = threadIdx.x; i < ldv; i += blockDim.x) g[i] = 0.0;
  if (threadIdx.x == 0) {
    const int on = active[p] != 0;
    st[p].done = !on;
    st[p].skip_apply = !on;
    st[p].finishing = 0;
    st[p].k = 0;
    st[p].nan = 0;
    st[p].est = 0.0;
    st[p].nu = 1.0;
    if (p == 0) {
      ctl->napply_left = nactive;
      ctl->ndone = npairs - nactive;
      ctl->skip_all_apply = nactive == 0;
      ctl->all_done = nactive == 0;
    }
  }
}

// Back substitution y = R(0:k,0:k)^{-1} g(0:k) for pair blockIdx.x, one
// wavefront: R is staged in LDS, each step finishes one unknown and updates
// the remaining right-hand side in parallel.
__global__ __launch_bounds__(64) void backsolve_kernel(const GmresState *__restrict__ st_all,
                                                       const double *__restrict__ Hr_all, int ldh, int m,
                                                       const double *__restrict__ g_all,
                                                       double *__restrict__ y_all, int ldv) {
  __shared__ double R[kMaxCols][kMaxCols + 1];
  __shared__ double rhs[kMaxCols];
  const int p = blockIdx.x;
  const int k = st_all[p].k, t = threadIdx.x;
  const double *Hr = Hr_all + static_cast<int64_t>(p) * ldh * m;
  const double *g = g_all + static_cast<int64_t>(p) * ldv;
  double *y = y_all + static_cast<int64_t>(p) * ldv;
  for (int c = 0; c < k; ++c)
    for (int i = t; i <= c; i += 64) R[i][c] = Hr[static_cast<int64_t>(c) * ldh + i];
  for (int i = t; i < k; i += 64) rhs[i] = g[i];
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const double yi = rhs[i] / R[i][i];
    __syncthreads();
    for (int r = t; r < i; r += 64) rhs[r] -= R[r][i] * yi;
    if (t == 0) y[i] = yi;
    __syncthreads();
  }
}

}  // namespace
}  // namespace mdp
