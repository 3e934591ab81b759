// Host-side CSR matrices (FP64) and the sparse algebra the setup needs.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <stdexcept>
#include <vector>

namespace mdp {

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

// Sort the column indices of every row (values follow); duplicate columns are
// summed in their stored order.
inline void sort_rows(HCsr &a) {
  std::vector<std::pair<int32_t, double>> tmp;
  HCsr out = HCsr::empty(a.nr, a.nc);
  out.col.reserve(a.col.size());
  out.val.reserve(a.val.size());
  for (int32_t i = 0; i < a.nr; ++i) {
    tmp.clear();
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) tmp.emplace_back(a.col[p], a.val[p]);
    std::stable_sort(tmp.begin(), tmp.end(),
                     [](const auto &x, const auto &y) { return x.first < y.first; });
    for (size_t k = 0; k < tmp.size(); ++k) {
      if (!out.col.empty() && static_cast<int64_t>(out.col.size()) > out.ptr[i] &&
          out.col.back() == tmp[k].first) {
        out.val.back() += tmp[k].second;
      } else {
        out.col.push_back(tmp[k].first);
        out.val.push_back(tmp[k].second);
      }
    }
    out.ptr[i + 1] = static_cast<int32_t>(out.col.size());
  }
  a = std::move(out);
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

// C = A * B (Gustavson row-by-row with a dense accumulator).  Each output
// entry sums a_ik * b_kj over A's row in stored order, then B's row in stored
// order.  Output columns sorted; entries that sum to exactly zero are dropped.
inline HCsr spgemm(const HCsr &a, const HCsr &b) {
  if (a.nc != b.nr) throw std::invalid_argument("spgemm shape mismatch");
  HCsr c = HCsr::empty(a.nr, b.nc);
  std::vector<int32_t> mark(static_cast<size_t>(b.nc), -1);
  std::vector<double> acc(static_cast<size_t>(b.nc), 0.0);
  std::vector<int32_t> cols;
  for (int32_t i = 0; i < a.nr; ++i) {
    cols.clear();
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      const int32_t k = a.col[p];
      const double av = a.val[p];
      for (int32_t q = b.ptr[k]; q < b.ptr[k + 1]; ++q) {
        const int32_t j = b.col[q];
        if (mark[j] != i) {
          mark[j] = i;
          acc[j] = av * b.val[q];
          cols.push_back(j);
        } else {
          acc[j] += av * b.val[q];
        }
      }
    }
    std::sort(cols.begin(), cols.end());
    for (int32_t j : cols) {
      if (acc[j] == 0.0) continue;
      c.col.push_back(j);
      c.val.push_back(acc[j]);
    }
    c.ptr[i + 1] = static_cast<int32_t>(c.col.size());
  }
  return c;
}

// C = A - B for matrices with sorted rows; entries present in only one operand
// keep their value (negated for B); entries in both become a - b.  Results
// that are exactly zero are dropped.
inline HCsr subtract(const HCsr &a, const HCsr &b) {
  if (a.nr != b.nr || a.nc != b.nc) throw std::invalid_argument("subtract shape mismatch");
  HCsr c = HCsr::empty(a.nr, a.nc);
  c.col.reserve(a.col.size() + b.col.size());
  c.val.reserve(a.col.size() + b.col.size());
  for (int32_t i = 0; i < a.nr; ++i) {
    int32_t p = a.ptr[i], pe = a.ptr[i + 1], q = b.ptr[i], qe = b.ptr[i + 1];
    while (p < pe || q < qe) {
      if (q >= qe || (p < pe && a.col[p] < b.col[q])) {
        c.col.push_back(a.col[p]);
        c.val.push_back(a.val[p]);
        ++p;
      } else if (p >= pe || b.col[q] < a.col[p]) {
        c.col.push_back(b.col[q]);
        c.val.push_back(-b.val[q]);
        ++q;
      } else {
        const double v = a.val[p] - b.val[q];
        if (v != 0.0) {
          c.col.push_back(a.col[p]);
          c.val.push_back(v);
        }
        ++p;
        ++q;
      }
    }
    c.ptr[i + 1] = static_cast<int32_t>(c.col.size());
  }
  return c;
}

inline std::vector<double> diagonal(const HCsr &a) {
  std::vector<double> d(static_cast<size_t>(std::min(a.nr, a.nc)), 0.0);
  for (int32_t i = 0; i < a.nr && i < a.nc; ++i)
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
      if (a.col[p] == i) d[i] += a.val[p];
  return d;
}

inline std::vector<double> l1_row_norms(const HCsr &a) {
  std::vector<double> d(static_cast<size_t>(a.nr), 0.0);
  for (int32_t i = 0; i < a.nr; ++i) {
    double s = 0.0;
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) s += std::fabs(a.val[p]);
    d[i] = s;
  }
  return d;
}

// Submatrix with the given row and column index lists (both ascending maps
// old -> new via colmap; colmap[c] = -1 drops the column).
inline HCsr extract(const HCsr &a, const std::vector<int32_t> &rows,
                    const std::vector<int32_t> &colmap, int32_t ncols) {
  HCsr s = HCsr::empty(static_cast<int32_t>(rows.size()), ncols);
  for (size_t r = 0; r < rows.size(); ++r) {
    const int32_t i = rows[r];
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      const int32_t c = colmap[a.col[p]];
      if (c >= 0) {
        s.col.push_back(c);
        s.val.push_back(a.val[p]);
      }
    }
    s.ptr[r + 1] = static_cast<int32_t>(s.col.size());
  }
  return s;
}

}  // namespace mdp
