// Host-side CSR matrices (FP64) and the sparse algebra the setup needs.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <stdexcept>
#include <climits>
#include <thread>
#include <vector>

namespace mdp {

// Worker threads for the host setup (MDP_SETUP_THREADS, default: all cores,
// at most 32).
inline int setup_workers() {
  static const int n = [] {
    const char *e = std::getenv("MDP_SETUP_THREADS");
    int t = e ? std::atoi(e) : static_cast<int>(std::thread::hardware_concurrency());
    return std::max(1, std::min(t, 32));
  }();
  return n;
}

// Split [0, n) into at most setup_workers() contiguous chunks and run
// f(begin, end, chunk) on each in its own thread.  With work (the prefix sums
// of a per-row cost, size n + 1) the chunks carry equal shares of the cost,
// else equal numbers of rows; below 8192 units of cost everything runs on the
// calling thread.  The chunking depends only on n and work.  f must not
// throw.
template <class F>
void parallel_chunks(int64_t n, F &&f, const std::vector<int64_t> *work = nullptr) {
  const int64_t total = work ? (*work)[static_cast<size_t>(n)] : n;
  const int T = static_cast<int>(std::min<int64_t>(total < 8192 ? 1 : setup_workers(), std::max<int64_t>(n, 1)));
  if (T == 1) {
    f(int64_t{0}, n, 0);
    return;
  }
  std::vector<int64_t> bound(static_cast<size_t>(T) + 1, n);
  bound[0] = 0;
  for (int t = 1; t < T; ++t) {
    if (work) {
      const int64_t target = total / T * t + total % T * t / T;
      bound[t] = std::lower_bound(work->begin(), work->begin() + n + 1, target) - work->begin();
    } else {
      bound[t] = std::min<int64_t>(n, t * ((n + T - 1) / T));
    }
    bound[t] = std::max(bound[t], bound[t - 1]);
  }
  std::vector<std::thread> th;
  for (int t = 0; t < T; ++t) {
    const int64_t b = bound[t], e = bound[t + 1];
    if (b >= e) continue;
    th.emplace_back([&f, b, e, t] { f(b, e, t); });
  }
  for (auto &x : th) x.join();
}

struct HCsr {
  int32_t nr = 0, nc = 0;
  std::vector<int32_t> ptr{0};
  std::vector<int32_t> col;
  std::vector<double> val;

  int64_t nnz() const { return static_cast<int64_t>(col.size()); }
  static HCsr empty(int32_t nr, int32_t nc) {
    HCsr m;
    m.nr = nr;
    m.nc = nc;
    m.ptr.assign(static_cast<size_t>(nr) + 1, 0);
    return m;
  }
};

// Build a matrix row by row in parallel: fn(i, chunk, cols, vals) appends the
// entries of row i.  Rows are computed independently, so the result does not
// depend on the number of threads.
template <class RowFn>
HCsr build_rows(int32_t nr, int32_t nc, RowFn &&fn, const std::vector<int64_t> *work = nullptr) {
  const int T = setup_workers();
  std::vector<std::vector<int32_t>> lc(static_cast<size_t>(T));
  std::vector<std::vector<double>> lv(static_cast<size_t>(T));
  std::vector<int32_t> cnt(static_cast<size_t>(nr), 0);
  std::vector<int64_t> first(static_cast<size_t>(T), -1);
  parallel_chunks(nr, [&](int64_t b, int64_t e, int t) {
    auto &C = lc[t];
    auto &V = lv[t];
    first[t] = b;
    for (int64_t i = b; i < e; ++i) {
      const size_t before = C.size();
      fn(static_cast<int32_t>(i), t, C, V);
      cnt[i] = static_cast<int32_t>(C.size() - before);
    }
  }, work);
  HCsr out = HCsr::empty(nr, nc);
  int64_t acc = 0;
  for (int32_t i = 0; i < nr; ++i) {
    acc += cnt[i];
    if (acc > INT32_MAX) throw std::length_error("matrix exceeds int32 indexing");
    out.ptr[i + 1] = static_cast<int32_t>(acc);
  }
  out.col.resize(static_cast<size_t>(acc));
  out.val.resize(static_cast<size_t>(acc));
  // each chunk's rows go to their place; the chunks are copied by threads
  // of their own when there is enough to copy
  auto place = [&](int t) {
    if (first[t] < 0) return;
    const int64_t off = out.ptr[first[t]];
    std::copy(lc[t].begin(), lc[t].end(), out.col.begin() + off);
    std::copy(lv[t].begin(), lv[t].end(), out.val.begin() + off);
  };
  if (T > 1 && acc >= (int64_t{1} << 16)) {
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) th.emplace_back(place, t);
    for (auto &x : th) x.join();
  } else {
    for (int t = 0; t < T; ++t) place(t);
  }
  return out;
}

// Build a matrix in two parallel passes over its rows, for rows that are
// cheap to form twice (merges): emit(i, put) calls put(col, val) for each
// entry of row i in order; the first pass only counts them, the second writes
// them in place.  The result does not depend on the number of threads.
template <class Emit>
HCsr build_rows_twice(int32_t nr, int32_t nc, Emit &&emit) {
  HCsr out = HCsr::empty(nr, nc);
  std::vector<int32_t> cnt(static_cast<size_t>(nr), 0);
  parallel_chunks(nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      int32_t c = 0;
      emit(static_cast<int32_t>(i), [&c](int32_t, double) { ++c; });
      cnt[i] = c;
    }
  });
  int64_t acc = 0;
  for (int32_t i = 0; i < nr; ++i) {
    acc += cnt[i];
    if (acc > INT32_MAX) throw std::length_error("matrix exceeds int32 indexing");
    out.ptr[i + 1] = static_cast<int32_t>(acc);
  }
  out.col.resize(static_cast<size_t>(acc));
  out.val.resize(static_cast<size_t>(acc));
  parallel_chunks(nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      int32_t q = out.ptr[i];
      emit(static_cast<int32_t>(i), [&](int32_t c, double v) {
        out.col[q] = c;
        out.val[q] = v;
        ++q;
      });
    }
  });
  return out;
}

// Sort the column indices of every row (values follow); duplicate columns are
// summed in their stored order.
// Rows whose columns already increase strictly are kept as they are.
inline void sort_rows(HCsr &a) {
  a = build_rows_twice(a.nr, a.nc, [&](int32_t i, auto &&put) {
    const int32_t p0 = a.ptr[i], p1 = a.ptr[i + 1];
    bool sorted = true;
    for (int32_t p = p0 + 1; p < p1 && sorted; ++p) sorted = a.col[p - 1] < a.col[p];
    if (sorted) {
      for (int32_t p = p0; p < p1; ++p) put(a.col[p], a.val[p]);
      return;
    }
    static thread_local std::vector<std::pair<int32_t, double>> row;
    row.clear();
    for (int32_t p = p0; p < p1; ++p) row.emplace_back(a.col[p], a.val[p]);
    std::stable_sort(row.begin(), row.end(), [](const auto &x, const auto &y) { return x.first < y.first; });
    for (size_t k = 0; k < row.size();) {
      double v = row[k].second;
      size_t m = k + 1;
      for (; m < row.size() && row[m].first == row[k].first; ++m) v += row[m].second;
      put(row[k].first, v);
      k = m;
    }
  });
}

inline HCsr transpose(const HCsr &a) {
  HCsr t = HCsr::empty(a.nc, a.nr);
  std::vector<int32_t> cnt(static_cast<size_t>(a.nc) + 1, 0);
  for (int32_t c : a.col) cnt[c + 1]++;
  for (int32_t j = 0; j < a.nc; ++j) cnt[j + 1] += cnt[j];
  t.ptr = cnt;
  t.col.resize(a.col.size());
  t.val.resize(a.val.size());
  std::vector<int32_t> next(cnt.begin(), cnt.end() - 1);
  for (int32_t i = 0; i < a.nr; ++i)
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      int32_t q = next[a.col[p]]++;
      t.col[q] = i;
      t.val[q] = a.val[p];
    }
  return t;  // rows of t come out sorted because i increases
}

// Greedy colouring for multicolour Gauss-Seidel: in natural order, node i
// takes the smallest colour not used by an already coloured neighbour in the
// pattern of a + a^T (diagonal and stored zeros excluded).  Returns the
// colour of each node.
inline std::vector<int32_t> greedy_colours(const HCsr &a) {
  const HCsr t = transpose(a);
  std::vector<int32_t> col(static_cast<size_t>(a.nr), -1);
  std::vector<int32_t> seen;  // seen[c] == i: colour c is used by a neighbour of i
  for (int32_t i = 0; i < a.nr; ++i) {
    for (const HCsr *m : {&a, &t})
      for (int32_t p = m->ptr[i]; p < m->ptr[i + 1]; ++p) {
        const int32_t j = m->col[p];
        if (j == i || col[j] < 0 || m->val[p] == 0.0) continue;
        if (static_cast<size_t>(col[j]) >= seen.size()) seen.resize(static_cast<size_t>(col[j]) + 1, -1);
        seen[col[j]] = i;
      }
    int32_t c = 0;
    while (static_cast<size_t>(c) < seen.size() && seen[c] == i) ++c;
    col[i] = c;
  }
  return col;
}

// A device implementation of spgemm that returns the same matrix bit for
// bit, installed (per thread) by the library around a set-up that may use the
// GPU; products of at least min_terms terms go to it, and to the host when it
// returns false.
struct ProductHook {
  bool (*fn)(const HCsr &a, const HCsr &b, HCsr &c, void *ctx) = nullptr;
  void *ctx = nullptr;
  int64_t min_terms = 0;
};
inline ProductHook &product_hook() {
  static thread_local ProductHook h;
  return h;
}

// C = A * B (Gustavson row-by-row with a dense accumulator).  Each output
// entry sums a_ik * b_kj over A's row in stored order, then B's row in stored
// order.  Output columns sorted; entries that sum to exactly zero are dropped.
// Rows are shared among the threads by their number of products.
inline HCsr spgemm(const HCsr &a, const HCsr &b) {
  if (a.nc != b.nr) throw std::invalid_argument("spgemm shape mismatch");
  const int T = setup_workers();
  std::vector<int64_t> work(static_cast<size_t>(a.nr) + 1, 0);
  for (int32_t i = 0; i < a.nr; ++i) {
    int64_t w = 1;
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) w += b.ptr[a.col[p] + 1] - b.ptr[a.col[p]];
    work[i + 1] = work[i] + w;
  }
  const ProductHook &hook = product_hook();
  if (hook.fn && work[a.nr] - a.nr >= hook.min_terms) {
    HCsr c;
    if (hook.fn(a, b, c, hook.ctx)) return c;
  }
  std::vector<std::vector<int32_t>> mark(static_cast<size_t>(T)), cols(static_cast<size_t>(T));
  std::vector<std::vector<double>> acc(static_cast<size_t>(T));
  return build_rows(a.nr, b.nc, [&](int32_t i, int t, std::vector<int32_t> &C, std::vector<double> &V) {
    auto &mk = mark[t];
    auto &ac = acc[t];
    auto &cl = cols[t];
    if (mk.empty()) {
      mk.assign(static_cast<size_t>(b.nc), -1);
      ac.assign(static_cast<size_t>(b.nc), 0.0);
    }
    cl.clear();
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      const int32_t k = a.col[p];
      const double av = a.val[p];
      for (int32_t q = b.ptr[k]; q < b.ptr[k + 1]; ++q) {
        const int32_t j = b.col[q];
        if (mk[j] != i) {
          mk[j] = i;
          ac[j] = av * b.val[q];
          cl.push_back(j);
        } else {
          ac[j] += av * b.val[q];
        }
      }
    }
    std::sort(cl.begin(), cl.end());
    for (int32_t j : cl) {
      if (ac[j] == 0.0) continue;
      C.push_back(j);
      V.push_back(ac[j]);
    }
  }, &work);
}

// C = A - B for matrices with sorted rows; entries present in only one operand
// keep their value (negated for B); entries in both become a - b.  Results
// that are exactly zero are dropped.
inline HCsr subtract(const HCsr &a, const HCsr &b) {
  if (a.nr != b.nr || a.nc != b.nc) throw std::invalid_argument("subtract shape mismatch");
  return build_rows_twice(a.nr, a.nc, [&](int32_t i, auto &&put) {
    int32_t p = a.ptr[i], pe = a.ptr[i + 1], q = b.ptr[i], qe = b.ptr[i + 1];
    while (p < pe || q < qe) {
      if (q >= qe || (p < pe && a.col[p] < b.col[q])) {
        put(a.col[p], a.val[p]);
        ++p;
      } else if (p >= pe || b.col[q] < a.col[p]) {
        put(b.col[q], -b.val[q]);
        ++q;
      } else {
        const double v = a.val[p] - b.val[q];
        if (v != 0.0) put(a.col[p], v);
        ++p;
        ++q;
      }
    }
  });
}

// a == a^T exactly, values included, for a square matrix whose rows are
// sorted without repeated columns: every entry (i, j, v) has its mirror
// (j, i, v), found by binary search in row j.
inline bool is_symmetric(const HCsr &a) {
  if (a.nr != a.nc) return false;
  std::vector<char> bad(static_cast<size_t>(setup_workers()), 0);
  parallel_chunks(a.nr, [&](int64_t b, int64_t e, int t) {
    for (int64_t i = b; i < e && !bad[t]; ++i)
      for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
        const int32_t j = a.col[p];
        const auto lo = a.col.begin() + a.ptr[j], hi = a.col.begin() + a.ptr[j + 1];
        const auto q = std::lower_bound(lo, hi, static_cast<int32_t>(i));
        if (q == hi || *q != i || a.val[static_cast<size_t>(q - a.col.begin())] != a.val[p]) {
          bad[t] = 1;
          break;
        }
      }
  });
  for (char c : bad)
    if (c) return false;
  return true;
}

inline std::vector<double> diagonal(const HCsr &a) {
  std::vector<double> d(static_cast<size_t>(std::min(a.nr, a.nc)), 0.0);
  parallel_chunks(std::min(a.nr, a.nc), [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i)
      for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
        if (a.col[p] == i) d[i] += a.val[p];
  });
  return d;
}

inline std::vector<double> l1_row_norms(const HCsr &a) {
  std::vector<double> d(static_cast<size_t>(a.nr), 0.0);
  parallel_chunks(a.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      double s = 0.0;
      for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) s += std::fabs(a.val[p]);
      d[i] = s;
    }
  });
  return d;
}

// Submatrix with the given row and column index lists (both ascending maps
// old -> new via colmap; colmap[c] = -1 drops the column).
inline HCsr extract(const HCsr &a, const std::vector<int32_t> &rows,
                    const std::vector<int32_t> &colmap, int32_t ncols) {
  return build_rows_twice(static_cast<int32_t>(rows.size()), ncols, [&](int32_t r, auto &&put) {
    const int32_t i = rows[r];
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      const int32_t c = colmap[a.col[p]];
      if (c >= 0) put(c, a.val[p]);
    }
  });
}

}  // namespace mdp
