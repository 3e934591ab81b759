// Sparse products of the set-up on the device (Section 3.3's Galerkin
// products A P_t, R A, (R A) P and eq. (7)'s A_OG D^-1 A_GO), with the host
// product's result bit for bit.
//
// The host product (spgemm) forms every term a_ik b_kj of a row in a fixed
// order (A's row in stored order, then B's row in stored order), keeps the
// first term of each column and adds the later ones to it in that order, and
// drops sums that are exactly zero.  The device follows the same definition
// in four steps:
//  1. expansion: one thread per entry of A writes its terms, in B's row order,
//     at its place in the row-major order of all terms (an exclusive scan of
//     the term counts), each with the key (row, column);
//  2. a stable radix sort by key, which keeps the terms of one (row, column)
//     in their order of step 1;
//  3. the first term of each run of equal keys sums its run left to right,
//     with separately rounded products and additions as on the host;
//  4. the non-zero sums are compacted and the row pointers found by binary
//     search over the (sorted) rows.
#include "dev_spgemm.hpp"

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <string>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "runtime.hpp"
#include "types.hpp"

namespace mdp {

namespace {

constexpr int64_t kMaxTerms = int64_t{1} << 29;  // device buffers of about 32 bytes per term

int bits_for(int64_t n) {  // bits that hold 0 .. n - 1
  int b = 1;
  while (b < 62 && (int64_t{1} << b) < n) ++b;
  return b;
}

unsigned grid_of(int64_t n) { return static_cast<unsigned>((n + kThreads - 1) / kThreads); }

__global__ __launch_bounds__(kThreads) void term_count_kernel(int64_t nnz, const int *__restrict__ acol,
                                                              const int *__restrict__ bptr,
                                                              int64_t *__restrict__ t) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (p < nnz) t[p] = bptr[acol[p] + 1] - bptr[acol[p]];
}

// Entry p of A (row i, column k) writes the terms a_ik b_kj of B's row k at
// pos[p] ... pos[p] + len - 1.
__global__ __launch_bounds__(kThreads) void expand_kernel(int nr, int64_t nnz, const int *__restrict__ aptr,
                                                          const int *__restrict__ acol,
                                                          const double *__restrict__ aval,
                                                          const int *__restrict__ bptr,
                                                          const int *__restrict__ bcol,
                                                          const double *__restrict__ bval,
                                                          const int64_t *__restrict__ pos, int cbits,
                                                          uint64_t *__restrict__ key, double *__restrict__ val) {
  const int64_t p = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (p >= nnz) return;
  // the row of entry p: aptr[lo] <= p < aptr[lo + 1]
  int lo = 0, hi = nr;
  while (hi - lo > 1) {
    const int mid = lo + (hi - lo) / 2;
    if (aptr[mid] <= p)
      lo = mid;
    else
      hi = mid;
  }
  const int k = acol[p];
  const double av = aval[p];
  const uint64_t rk = static_cast<uint64_t>(lo) << cbits;
  int64_t o = pos[p];
  for (int q = bptr[k]; q < bptr[k + 1]; ++q, ++o) {
    key[o] = rk | static_cast<uint32_t>(bcol[q]);
    val[o] = av * bval[q];
  }
}

// The first term of each run of equal keys sums the run in order; flag = 1
// for runs whose sum is not exactly zero.
__global__ __launch_bounds__(kThreads) void run_sum_kernel(int64_t m, const uint64_t *__restrict__ key,
                                                           const double *__restrict__ val,
                                                           double *__restrict__ sum, uint32_t *__restrict__ flag) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= m) return;
  uint32_t f = 0;
  if (k == 0 || key[k] != key[k - 1]) {
    const uint64_t kk = key[k];
    double s = val[k];
    for (int64_t j = k + 1; j < m && key[j] == kk; ++j) s += val[j];
    sum[k] = s;
    f = s != 0.0;
  }
  flag[k] = f;
}

__global__ __launch_bounds__(kThreads) void scatter_kernel(int64_t m, const uint64_t *__restrict__ key,
                                                           const double *__restrict__ sum,
                                                           const uint32_t *__restrict__ flag,
                                                           const uint32_t *__restrict__ idx, int cbits,
                                                           int *__restrict__ ocol, double *__restrict__ oval,
                                                           int *__restrict__ orow) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (k >= m || !flag[k]) return;
  const uint32_t o = idx[k];
  const uint64_t kk = key[k];
  ocol[o] = static_cast<int>(kk & ((uint64_t{1} << cbits) - 1));
  orow[o] = static_cast<int>(kk >> cbits);
  oval[o] = sum[k];
}

// optr[i] = the number of output entries in rows before i.
__global__ __launch_bounds__(kThreads) void row_ptr_kernel(int nr, int64_t u, const int *__restrict__ orow,
                                                           int *__restrict__ optr) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x;
  if (i > nr) return;
  int64_t lo = 0, hi = u;  // first index with orow >= i
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo) / 2;
    if (orow[mid] < i)
      lo = mid + 1;
    else
      hi = mid;
  }
  optr[i] = static_cast<int>(lo);
}

template <typename V>
void put(DevMem &d, const std::vector<V> &h, hipStream_t s) {
  d.alloc(std::max<size_t>(h.size(), 1) * sizeof(V));
  if (!h.empty()) MDP_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, s));
}

}  // namespace

bool device_spgemm(const HCsr &a, const HCsr &b, HCsr &c, void *stream) {
  if (a.nc != b.nr) throw std::invalid_argument("spgemm shape mismatch");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int64_t nnz = a.nnz();
  int64_t m = 0;
  for (int64_t p = 0; p < nnz; ++p) m += b.ptr[a.col[p] + 1] - b.ptr[a.col[p]];
  if (nnz == 0 || m == 0 || m > kMaxTerms || a.nr <= 0 || b.nc <= 0) return false;
  const int cbits = bits_for(b.nc), rbits = bits_for(a.nr);
  if (cbits + rbits > 64) return false;
  const bool verbose = std::getenv("MDP_SETUP_VERBOSE") != nullptr;
  auto t_prev = std::chrono::steady_clock::now();
  char lapbuf[256];
  std::string laps;
  auto lap = [&](const char *what) {
    if (!verbose) return;
    MDP_HIP(hipStreamSynchronize(s));
    const auto now = std::chrono::steady_clock::now();
    std::snprintf(lapbuf, sizeof lapbuf, " %s %.1f", what, 1e3 * std::chrono::duration<double>(now - t_prev).count());
    laps += lapbuf;
    t_prev = now;
  };
  try {
    DevMem aptr, acol, aval, bptr, bcol, bval, pos, key0, key1, val0, val1;
    put(aptr, a.ptr, s);
    put(acol, a.col, s);
    put(aval, a.val, s);
    put(bptr, b.ptr, s);
    put(bcol, b.col, s);
    put(bval, b.val, s);
    lap("upload");
    // term counts per entry of A, then their exclusive scan (in key1's space)
    pos.alloc(sizeof(int64_t) * nnz);
    key1.alloc(sizeof(uint64_t) * std::max<int64_t>(m, nnz));
    int64_t *cnt = dptr<int64_t>(key1);
    hipLaunchKernelGGL(term_count_kernel, dim3(grid_of(nnz)), dim3(kThreads), 0, s, nnz, dptr<const int>(acol),
                       dptr<const int>(bptr), cnt);
    MDP_HIP(hipGetLastError());
    size_t tmp_bytes = 0;
    MDP_HIP(rocprim::exclusive_scan(nullptr, tmp_bytes, cnt, dptr<int64_t>(pos), int64_t{0},
                                    static_cast<size_t>(nnz), rocprim::plus<int64_t>(), s));
    DevMem tmp(std::max<size_t>(tmp_bytes, 1));
    MDP_HIP(rocprim::exclusive_scan(tmp.get(), tmp_bytes, cnt, dptr<int64_t>(pos), int64_t{0},
                                    static_cast<size_t>(nnz), rocprim::plus<int64_t>(), s));
    int64_t last[2] = {0, 0};
    MDP_HIP(hipMemcpyAsync(&last[0], dptr<int64_t>(pos) + (nnz - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MDP_HIP(hipMemcpyAsync(&last[1], cnt + (nnz - 1), sizeof(int64_t), hipMemcpyDeviceToHost, s));
    MDP_HIP(hipStreamSynchronize(s));
    if (last[0] + last[1] != m) raise(MDP_EHIP, "device product: term count mismatch");
    lap("scan");
    // 1. expansion
    key0.alloc(sizeof(uint64_t) * m);
    val0.alloc(sizeof(double) * m);
    val1.alloc(sizeof(double) * m);
    hipLaunchKernelGGL(expand_kernel, dim3(grid_of(nnz)), dim3(kThreads), 0, s, a.nr, nnz, dptr<const int>(aptr),
                       dptr<const int>(acol), dptr<const double>(aval), dptr<const int>(bptr),
                       dptr<const int>(bcol), dptr<const double>(bval), dptr<const int64_t>(pos), cbits,
                       dptr<uint64_t>(key0), dptr<double>(val0));
    MDP_HIP(hipGetLastError());
    lap("alloc+expand");
    // 2. stable sort by (row, column): key0/val0 -> key1/val1
    const unsigned end_bit = static_cast<unsigned>(cbits + rbits);
    size_t sort_bytes = 0;
    MDP_HIP(rocprim::radix_sort_pairs(nullptr, sort_bytes, dptr<uint64_t>(key0), dptr<uint64_t>(key1),
                                      dptr<double>(val0), dptr<double>(val1), static_cast<size_t>(m), 0u, end_bit,
                                      s));
    DevMem sort_tmp(std::max<size_t>(sort_bytes, 1));
    MDP_HIP(rocprim::radix_sort_pairs(sort_tmp.get(), sort_bytes, dptr<uint64_t>(key0), dptr<uint64_t>(key1),
                                      dptr<double>(val0), dptr<double>(val1), static_cast<size_t>(m), 0u, end_bit,
                                      s));
    sort_tmp.reset();
    lap("sort");
    // 3. run sums (into val0) and their non-zero flags, then the flags'
    // exclusive scan (flags and indices in key0's space)
    uint32_t *flag = dptr<uint32_t>(key0), *idx = flag + m;
    hipLaunchKernelGGL(run_sum_kernel, dim3(grid_of(m)), dim3(kThreads), 0, s, m, dptr<const uint64_t>(key1),
                       dptr<const double>(val1), dptr<double>(val0), flag);
    MDP_HIP(hipGetLastError());
    size_t scan_bytes = 0;
    MDP_HIP(rocprim::exclusive_scan(nullptr, scan_bytes, flag, idx, uint32_t{0}, static_cast<size_t>(m),
                                    rocprim::plus<uint32_t>(), s));
    DevMem scan_tmp(std::max<size_t>(scan_bytes, 1));
    MDP_HIP(rocprim::exclusive_scan(scan_tmp.get(), scan_bytes, flag, idx, uint32_t{0}, static_cast<size_t>(m),
                                    rocprim::plus<uint32_t>(), s));
    uint32_t tail[2] = {0, 0};
    MDP_HIP(hipMemcpyAsync(&tail[0], idx + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    MDP_HIP(hipMemcpyAsync(&tail[1], flag + (m - 1), sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    MDP_HIP(hipStreamSynchronize(s));
    const int64_t u = static_cast<int64_t>(tail[0]) + tail[1];
    lap("sums");
    if (u > INT32_MAX) throw std::length_error("matrix exceeds int32 indexing");
    // 4. compaction and row pointers
    DevMem ocol(sizeof(int) * std::max<int64_t>(u, 1)), oval(sizeof(double) * std::max<int64_t>(u, 1)),
        orow(sizeof(int) * std::max<int64_t>(u, 1)), optr(sizeof(int) * (static_cast<size_t>(a.nr) + 1));
    hipLaunchKernelGGL(scatter_kernel, dim3(grid_of(m)), dim3(kThreads), 0, s, m, dptr<const uint64_t>(key1),
                       dptr<const double>(val0), flag, idx, cbits, dptr<int>(ocol), dptr<double>(oval),
                       dptr<int>(orow));
    MDP_HIP(hipGetLastError());
    hipLaunchKernelGGL(row_ptr_kernel, dim3(grid_of(static_cast<int64_t>(a.nr) + 1)), dim3(kThreads), 0, s, a.nr,
                       u, dptr<const int>(orow), dptr<int>(optr));
    MDP_HIP(hipGetLastError());
    lap("compact");
    c = HCsr::empty(a.nr, b.nc);
    c.col.resize(static_cast<size_t>(u));
    c.val.resize(static_cast<size_t>(u));
    MDP_HIP(hipMemcpyAsync(c.ptr.data(), optr.get(), sizeof(int) * (static_cast<size_t>(a.nr) + 1),
                           hipMemcpyDeviceToHost, s));
    if (u > 0) {
      MDP_HIP(hipMemcpyAsync(c.col.data(), ocol.get(), sizeof(int) * u, hipMemcpyDeviceToHost, s));
      MDP_HIP(hipMemcpyAsync(c.val.data(), oval.get(), sizeof(double) * u, hipMemcpyDeviceToHost, s));
    }
    MDP_HIP(hipStreamSynchronize(s));
    lap("download");
    if (verbose)
      std::fprintf(stderr, "[mdp] device product %d x %d, %lld terms -> %lld: ms%s\n", a.nr, b.nc,
                   static_cast<long long>(m), static_cast<long long>(u), laps.c_str());
    return true;
  } catch (const Error &e) {
    if (e.code != MDP_ENOMEM) throw;
    (void)hipGetLastError();  // clear the failed allocation's error state
    return false;
  }
}

}  // namespace mdp
