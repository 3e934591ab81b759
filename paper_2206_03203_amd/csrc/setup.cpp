// Host setup: validation, [Omega; Gamma] split (eq. 4), S~ (eq. 7) and the
// smoothed-aggregation hierarchies that define Q_OO and Q_GG (Section 3.3).
//
// SA-AMG rules (the paper names SA-AMG but leaves its parameters open):
//  * strength: j != i strong for i iff |a_ij| >= theta sqrt(|a_ii a_jj|);
//  * greedy aggregation in natural order, three passes: (1) a node whose
//    strong neighbourhood is entirely free (itself included) seeds an
//    aggregate with it; (2) free nodes join the first-pass aggregate of their
//    lowest-numbered strong neighbour that the first pass placed; (3) nodes
//    still free seed aggregates with their still-free strong neighbours.
//    Nodes without strong neighbours stay out (zero tentative row);
//  * tentative prolongator columns = aggregate indicators / sqrt(size);
//  * P = P_t - omega D^{-1} A P_t, D = diag(A), omega = 4 / (3 rho),
//    rho = max_i sum_j |a_ij| / |a_ii| (Gershgorin bound of D^{-1} A);
//  * R = P^T, A_c = (R A) P;
//  * stop at n <= max_coarse, no aggregate, n_c > 0.9 n, or max_levels;
//  * coarsest: dense LU inverse if n <= max_dense, else l1-Jacobi sweeps.
#include "setup.hpp"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <limits>
#include <numeric>

namespace mdp {

namespace {

[[noreturn]] void fail(int code, const std::string &msg) { throw SetupError{code, msg}; }

// Phase timings on stderr when MDP_SETUP_VERBOSE is set.
struct PhaseClock {
  bool on = std::getenv("MDP_SETUP_VERBOSE") != nullptr;
  std::chrono::steady_clock::time_point t = std::chrono::steady_clock::now();
  void lap(const char *what) {
    if (!on) return;
    const auto now = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[mdp setup] %-28s %8.3f s\n", what, std::chrono::duration<double>(now - t).count());
    t = now;
  }
};

void validate(const mdp_csr *A, const int32_t *part) {
  if (!A || !part) fail(MDP_EINVAL, "NULL matrix or partition");
  if (A->n <= 0) fail(MDP_EINVAL, "n must be positive");
  if (!A->row_ptr || (A->nnz > 0 && (!A->col || !A->val))) fail(MDP_EINVAL, "NULL CSR array");
  if (A->nnz < 0 || A->nnz > std::numeric_limits<int32_t>::max())
    fail(MDP_EINVAL, "nnz out of range (int32 indices)");
  if (A->row_ptr[0] != 0) fail(MDP_EINVAL, "row_ptr[0] must be 0");
  for (int32_t i = 0; i < A->n; ++i)
    if (A->row_ptr[i + 1] < A->row_ptr[i]) fail(MDP_EINVAL, "row_ptr is not non-decreasing");
  if (A->row_ptr[A->n] != A->nnz) fail(MDP_EINVAL, "row_ptr[n] != nnz");
  for (int64_t p = 0; p < A->nnz; ++p) {
    if (A->col[p] < 0 || A->col[p] >= A->n) fail(MDP_EINVAL, "column index out of range");
    if (!std::isfinite(A->val[p])) fail(MDP_ENAN, "non-finite matrix value");
  }
  for (int32_t i = 0; i < A->n; ++i)
    if (part[i] != 0 && part[i] != 1) fail(MDP_EINVAL, "part entries must be 0 or 1");
}

void check_diag(const HCsr &a, const char *what) {
  std::vector<double> d = diagonal(a);
  for (size_t i = 0; i < d.size(); ++i)
    if (!(d[i] > 0.0))
      fail(MDP_ENONPOS_DIAG, std::string("non-positive diagonal in ") + what + " at row " +
                                 std::to_string(i));
}

// Strong neighbours of every row as a CSR pattern (ascending columns); with
// labels (dimension-aware aggregation), only neighbours of the same label.
void strength(const HCsr &a, double theta, const int32_t *labels, std::vector<int32_t> &sp,
              std::vector<int32_t> &sc) {
  const std::vector<double> d = diagonal(a);
  // two parallel passes over the rows: count the strong neighbours, then
  // write them at their row offsets
  auto strong = [&](int32_t i, int32_t p) {
    const int32_t j = a.col[p];
    if (j == i || (labels && labels[j] != labels[i])) return false;
    return std::fabs(a.val[p]) >= theta * std::sqrt(std::fabs(d[i] * d[j]));
  };
  sp.assign(static_cast<size_t>(a.nr) + 1, 0);
  parallel_chunks(a.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      int32_t c = 0;
      for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) c += strong(static_cast<int32_t>(i), p);
      sp[i + 1] = c;
    }
  });
  for (int32_t i = 0; i < a.nr; ++i) sp[i + 1] += sp[i];
  sc.resize(static_cast<size_t>(sp[a.nr]));
  parallel_chunks(a.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      int32_t q = sp[i];
      for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p)
        if (strong(static_cast<int32_t>(i), p)) sc[q++] = a.col[p];
    }
  });
}

int32_t aggregate(int32_t n, const std::vector<int32_t> &sp, const std::vector<int32_t> &sc,
                  std::vector<int32_t> &agg) {
  agg.assign(static_cast<size_t>(n), -1);
  int32_t na = 0;
  for (int32_t i = 0; i < n; ++i) {  // first pass: free neighbourhoods
    if (sp[i] == sp[i + 1] || agg[i] != -1) continue;
    bool free = true;
    for (int32_t p = sp[i]; p < sp[i + 1] && free; ++p) free = agg[sc[p]] == -1;
    if (!free) continue;
    agg[i] = na;
    for (int32_t p = sp[i]; p < sp[i + 1]; ++p) agg[sc[p]] = na;
    ++na;
  }
  const std::vector<int32_t> first(agg);
  for (int32_t i = 0; i < n; ++i) {  // second pass: attach to first-pass aggregates
    if (agg[i] != -1 || sp[i] == sp[i + 1]) continue;
    for (int32_t p = sp[i]; p < sp[i + 1]; ++p)
      if (first[sc[p]] != -1) {
        agg[i] = first[sc[p]];
        break;
      }
  }
  for (int32_t i = 0; i < n; ++i) {  // third pass: leftovers
    if (agg[i] != -1 || sp[i] == sp[i + 1]) continue;
    agg[i] = na;
    for (int32_t p = sp[i]; p < sp[i + 1]; ++p)
      if (agg[sc[p]] == -1) agg[sc[p]] = na;
    ++na;
  }
  return na;
}

HCsr tentative(const std::vector<int32_t> &agg, int32_t na) {
  const int32_t n = static_cast<int32_t>(agg.size());
  std::vector<int32_t> size(static_cast<size_t>(na), 0);
  for (int32_t a : agg)
    if (a >= 0) size[a]++;
  HCsr t = HCsr::empty(n, na);
  for (int32_t i = 0; i < n; ++i) {
    if (agg[i] >= 0) {
      t.col.push_back(agg[i]);
      t.val.push_back(1.0 / std::sqrt(static_cast<double>(size[agg[i]])));
    }
    t.ptr[i + 1] = static_cast<int32_t>(t.col.size());
  }
  return t;
}

HCsr smooth_prolongator(const HCsr &a, const HCsr &pt) {
  const std::vector<double> d = diagonal(a);
  const std::vector<double> l1 = l1_row_norms(a);
  double rho = 0.0;
  for (int32_t i = 0; i < a.nr; ++i) rho = std::max(rho, l1[i] / std::fabs(d[i]));
  const double omega = (4.0 / 3.0) / rho;
  HCsr ap = spgemm(a, pt);
  parallel_chunks(ap.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i)
      for (int32_t p = ap.ptr[i]; p < ap.ptr[i + 1]; ++p) ap.val[p] = omega * ((1.0 / d[i]) * ap.val[p]);
  });
  return subtract(pt, ap);
}

// Dense inverse by LU with partial pivoting (row-major, n x n).
std::vector<double> dense_inverse(const HCsr &a) {
  const int32_t n = a.nr;
  std::vector<double> m(static_cast<size_t>(n) * n, 0.0), inv(static_cast<size_t>(n) * n, 0.0);
  double amax = 0.0;
  for (int32_t i = 0; i < n; ++i)
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
      m[static_cast<size_t>(i) * n + a.col[p]] += a.val[p];
      amax = std::max(amax, std::fabs(a.val[p]));
    }
  for (int32_t i = 0; i < n; ++i) inv[static_cast<size_t>(i) * n + i] = 1.0;
  const double tiny = amax * std::numeric_limits<double>::epsilon() * n;
  for (int32_t k = 0; k < n; ++k) {
    int32_t piv = k;
    double best = std::fabs(m[static_cast<size_t>(k) * n + k]);
    for (int32_t i = k + 1; i < n; ++i) {
      const double v = std::fabs(m[static_cast<size_t>(i) * n + k]);
      if (v > best) {
        best = v;
        piv = i;
      }
    }
    if (!(best > tiny)) fail(MDP_ESINGULAR, "coarsest level is singular to working precision");
    if (piv != k)
      for (int32_t j = 0; j < n; ++j) {
        std::swap(m[static_cast<size_t>(k) * n + j], m[static_cast<size_t>(piv) * n + j]);
        std::swap(inv[static_cast<size_t>(k) * n + j], inv[static_cast<size_t>(piv) * n + j]);
      }
    const double dk = m[static_cast<size_t>(k) * n + k];
    for (int32_t i = 0; i < n; ++i) {
      if (i == k) continue;
      const double f = m[static_cast<size_t>(i) * n + k] / dk;
      if (f == 0.0) continue;
      double *ri = &m[static_cast<size_t>(i) * n];
      const double *rk = &m[static_cast<size_t>(k) * n];
      for (int32_t j = k; j < n; ++j) ri[j] -= f * rk[j];
      double *qi = &inv[static_cast<size_t>(i) * n];
      const double *qk = &inv[static_cast<size_t>(k) * n];
      for (int32_t j = 0; j < n; ++j) qi[j] -= f * qk[j];
    }
    double *rk = &m[static_cast<size_t>(k) * n];
    double *qk = &inv[static_cast<size_t>(k) * n];
    for (int32_t j = k; j < n; ++j) rk[j] /= dk;
    for (int32_t j = 0; j < n; ++j) qk[j] /= dk;
  }
  for (double v : inv)
    if (!std::isfinite(v)) fail(MDP_ESINGULAR, "coarsest inverse is not finite");
  return inv;
}

// For a matrix with non-positive off-diagonals (an M-matrix candidate, as
// two-point flux produces; symmetric or not), call row i grounded when its
// row sum is positive (a Dirichlet contact).  The rows that cannot reach a
// grounded row along their nonzeros (i -> j for a_ij != 0) form a set U
// closed under that relation whose rows all sum to zero, so A[U, U] 1 = 0 and
// the rows of U couple only to U: A is singular, nothing ties the level of
// U.  Such input cannot be solved and is rejected up front.
void check_grounded(const HCsr &a, bool symmetric) {
  const int32_t n = a.nr;
  std::vector<double> rs(static_cast<size_t>(n), 0.0), dg(static_cast<size_t>(n), 0.0);
  std::vector<char> positive(static_cast<size_t>(setup_workers()), 0);
  parallel_chunks(n, [&](int64_t b, int64_t e, int t) {
    for (int64_t i = b; i < e && !positive[t]; ++i)
      for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) {
        if (a.col[p] != i && a.val[p] > 0.0) {
          positive[t] = 1;
          break;
        }
        rs[i] += a.val[p];
        if (a.col[p] == i) dg[i] = a.val[p];
      }
  });
  for (char c : positive)
    if (c) return;  // not an M-matrix pattern: no claim
  // walk the transpose from the grounded rows: row j reaches ground when
  // a_ji != 0 for a row i that does
  const HCsr tt = symmetric ? HCsr::empty(0, 0) : transpose(a);
  const HCsr &t = symmetric ? a : tt;
  std::vector<char> reach(static_cast<size_t>(n), 0);
  std::vector<int32_t> stack;
  for (int32_t i = 0; i < n; ++i)
    if (rs[i] > 1e-10 * dg[i]) {
      reach[i] = 1;
      stack.push_back(i);
    }
  while (!stack.empty()) {
    const int32_t i = stack.back();
    stack.pop_back();
    for (int32_t p = t.ptr[i]; p < t.ptr[i + 1]; ++p) {  // rows j with a_ji != 0
      const int32_t j = t.col[p];
      if (t.val[p] != 0.0 && !reach[j]) {
        reach[j] = 1;
        stack.push_back(j);
      }
    }
  }
  for (int32_t i = 0; i < n; ++i)
    if (!reach[i])
      fail(MDP_ESINGULAR, "row " + std::to_string(i) +
                              " cannot reach a row with a positive row sum: no boundary condition fixes the level "
                              "of the unknowns it couples to");
}

}  // namespace

// The V-cycle's residual after its first smoothing iterate x0 = D^-1 b is
// b - A D^-1 b, and only its restriction is used: R (I - A D^-1) b.  That
// matrix, from the R A already formed for the Galerkin product, restricts b
// in one product instead of two dependent ones (the operator is the same; the
// rounding differs).  It is kept only when that product moves no more bytes
// than the two it replaces (8-byte values, 4-byte indices).
HCsr fused_restriction(const HLevel &L, const HCsr &ra) {
  // R - (R A) D^-1, row by row in parallel: a merge of the two sorted rows,
  // the (R A) entries divided by the l1 diagonal of their column
  const HCsr &r = L.R;
  const std::vector<double> &d = L.dl1;
  if (r.nr != ra.nr || r.nc != ra.nc) throw std::invalid_argument("fused restriction shape mismatch");
  HCsr f = build_rows_twice(r.nr, r.nc, [&](int32_t i, auto &&put) {
    int32_t p = r.ptr[i], pe = r.ptr[i + 1], q = ra.ptr[i], qe = ra.ptr[i + 1];
    while (p < pe || q < qe) {
      if (q >= qe || (p < pe && r.col[p] < ra.col[q])) {
        put(r.col[p], r.val[p]);
        ++p;
      } else if (p >= pe || ra.col[q] < r.col[p]) {
        put(ra.col[q], -(ra.val[q] / d[static_cast<size_t>(ra.col[q])]));
        ++q;
      } else {
        const double v = r.val[p] - ra.val[q] / d[static_cast<size_t>(ra.col[q])];
        if (v != 0.0) put(r.col[p], v);
        ++p;
        ++q;
      }
    }
  });
  const double n = L.A.nr, nc = L.R.nr;
  const double two = 12.0 * static_cast<double>(L.A.nnz() + L.R.nnz()) + 8.0 * (4.0 * n + 2.0 * nc);
  const double one = 12.0 * static_cast<double>(f.nnz()) + 8.0 * (n + 2.0 * nc);
  return one <= two ? f : HCsr::empty(0, 0);
}

namespace {

void csr_mv(const HCsr &a, const double *x, double *y) {
  for (int32_t i = 0; i < a.nr; ++i) {
    double acc = 0.0;
    for (int32_t p = a.ptr[i]; p < a.ptr[i + 1]; ++p) acc += a.val[p] * x[a.col[p]];
    y[i] = acc;
  }
}

// Work vectors of one thread, per level.
struct TailScratch {
  std::vector<std::vector<double>> ax, bc, xc;
};

// x = one V-cycle from zero on levels l.. of h (Section 3.3), in FP64 and in
// the steps the device takes with l1-Jacobi smoothing: the first iterate
// D^-1 b and pre - 1 further sweeps, the residual restricted by R, the coarse
// correction added through P, post sweeps; the coarsest level's dense inverse.
void vcycle_from(const HHier &h, size_t l, const double *b, double *x, int pre, int post, TailScratch &s) {
  const HLevel &L = h.lv[l];
  const int32_t n = L.A.nr;
  if (l + 1 == h.lv.size()) {
    for (int32_t i = 0; i < n; ++i) {
      double acc = 0.0;
      const double *row = h.coarse_inv.data() + static_cast<size_t>(i) * n;
      for (int32_t j = 0; j < n; ++j) acc += row[j] * b[j];
      x[i] = acc;
    }
    return;
  }
  double *ax = s.ax[l].data(), *bc = s.bc[l].data(), *xc = s.xc[l].data();
  for (int32_t i = 0; i < n; ++i) x[i] = b[i] / L.dl1[i];
  for (int k = 1; k < pre; ++k) {
    csr_mv(L.A, x, ax);
    for (int32_t i = 0; i < n; ++i) x[i] += (b[i] - ax[i]) / L.dl1[i];
  }
  csr_mv(L.A, x, ax);
  for (int32_t i = 0; i < n; ++i) ax[i] = b[i] - ax[i];
  csr_mv(L.R, ax, bc);
  vcycle_from(h, l + 1, bc, xc, pre, post, s);
  csr_mv(L.P, xc, ax);
  for (int32_t i = 0; i < n; ++i) x[i] += ax[i];
  for (int k = 0; k < post; ++k) {
    csr_mv(L.A, x, ax);
    for (int32_t i = 0; i < n; ++i) x[i] += (b[i] - ax[i]) / L.dl1[i];
  }
}

}  // namespace

void clear_tail(HHier &h) {
  h.tail = -1;
  h.tail_pre = h.tail_post = h.tail_max = 0;
  h.tail_op.clear();
}

// The V-cycle is linear in b (fixed sweeps from zero, a fixed coarse solve),
// so its part from level `tail` down is a matrix: column j is the V-cycle of
// the unit vector e_j.  Columns are formed independently on the set-up
// threads, so the matrix does not depend on their number.
void form_tail(HHier &h, int pre, int post, int32_t max_n) {
  if (h.tail_max == max_n && h.tail_pre == pre && h.tail_post == post && (h.tail >= 0 || h.tail_max > 0)) return;
  clear_tail(h);
  h.tail_pre = pre;
  h.tail_post = post;
  h.tail_max = max_n;
  if (!h.dense || h.lv.size() < 3) return;
  size_t ls = 0;
  for (size_t l = 1; l + 1 < h.lv.size(); ++l)
    if (h.lv[l].A.nr <= max_n) {
      ls = l;
      break;
    }
  if (ls == 0) return;
  const int32_t n = h.lv[ls].A.nr;
  int64_t per_col = 1;
  for (size_t l = ls; l < h.lv.size(); ++l)
    per_col += h.lv[l].A.nnz() * (pre + post + 1) + h.lv[l].R.nnz() + h.lv[l].P.nnz();
  per_col += static_cast<int64_t>(h.lv.back().A.nr) * h.lv.back().A.nr;
  std::vector<int64_t> work(static_cast<size_t>(n) + 1);
  for (int32_t j = 0; j <= n; ++j) work[j] = per_col * j;
  std::vector<double> T(static_cast<size_t>(n) * n);
  std::vector<TailScratch> scratch(static_cast<size_t>(setup_workers()));
  parallel_chunks(n, [&](int64_t b, int64_t e, int t) {
    TailScratch &sc = scratch[t];
    sc.ax.resize(h.lv.size());
    sc.bc.resize(h.lv.size());
    sc.xc.resize(h.lv.size());
    for (size_t l = ls; l + 1 < h.lv.size(); ++l) {
      sc.ax[l].assign(static_cast<size_t>(h.lv[l].A.nr), 0.0);
      sc.bc[l].assign(static_cast<size_t>(h.lv[l + 1].A.nr), 0.0);
      sc.xc[l].assign(static_cast<size_t>(h.lv[l + 1].A.nr), 0.0);
    }
    std::vector<double> ej(static_cast<size_t>(n), 0.0), col(static_cast<size_t>(n));
    for (int64_t j = b; j < e; ++j) {
      ej[j] = 1.0;
      vcycle_from(h, ls, ej.data(), col.data(), pre, post, sc);
      ej[j] = 0.0;
      for (int32_t i = 0; i < n; ++i) T[static_cast<size_t>(i) * n + j] = col[i];
    }
  }, &work);
  for (double v : T)
    if (!std::isfinite(v)) return;  // keep the levels themselves
  h.tail = static_cast<int32_t>(ls);
  h.tail_op = std::move(T);
}

HHier amg_setup(const HCsr &A, const AmgParams &prm, const int32_t *labels) {
  PhaseClock clk;
  HHier h;
  HCsr cur = A;
  std::vector<int32_t> sp, sc;
  while (true) {
    HLevel lv;
    lv.A = std::move(cur);
    lv.dl1 = l1_row_norms(lv.A);
    const int32_t n = lv.A.nr;
    h.lv.push_back(std::move(lv));
    HLevel &L = h.lv.back();
    if (n <= prm.max_coarse || static_cast<int32_t>(h.lv.size()) >= prm.max_levels) break;
    // dimension-aware aggregation (Section 3.3): aggregates of the finest
    // level stay inside one label; coarser levels may cross labels
    strength(L.A, prm.theta, h.lv.size() == 1 ? labels : nullptr, sp, sc);
    clk.lap("strength");
    std::vector<int32_t> agg;
    const int32_t na = aggregate(n, sp, sc, agg);
    clk.lap("aggregate");
    if (na == 0 || na > 0.9 * n) break;
    L.P = smooth_prolongator(L.A, tentative(agg, na));
    clk.lap("prolongator");
    L.R = transpose(L.P);
    L.agg = std::move(agg);
    clk.lap("transpose");
    HCsr ra = spgemm(L.R, L.A);
    clk.lap("R A");
    L.Rf = fused_restriction(L, ra);
    clk.lap("R (I - A D^-1)");
    cur = spgemm(ra, L.P);
    clk.lap("(R A) P");
  }
  const HLevel &last = h.lv.back();
  if (last.A.nr <= prm.max_dense) {
    h.dense = true;
    h.coarse_inv = dense_inverse(last.A);
  }
  clk.lap("coarsest inverse");
  return h;
}

void build_host_system(const mdp_csr *Ain, const int32_t *part, const mdp_options &opt,
                       HostSystem &s, const int32_t *label) {
  PhaseClock clk;
  validate(Ain, part);
  clk.lap("validate");
  const int32_t n = Ain->n;
  s.n = n;
  s.perm.clear();
  for (int32_t i = 0; i < n; ++i)
    if (part[i] == 0) s.perm.push_back(i);
  s.n_o = static_cast<int32_t>(s.perm.size());
  for (int32_t i = 0; i < n; ++i)
    if (part[i] == 1) s.perm.push_back(i);
  s.n_g = n - s.n_o;
  if (s.n_o == 0) fail(MDP_EINVAL, "no host-domain (part 0) unknowns");
  std::vector<int32_t> inv(static_cast<size_t>(n));
  s.identity = true;
  for (int32_t r = 0; r < n; ++r) {
    inv[s.perm[r]] = r;
    if (s.perm[r] != r) s.identity = false;
  }

  HCsr A = build_rows_twice(n, n, [&](int32_t r, auto &&put) {
    const int32_t i = s.perm[r];
    for (int32_t p = Ain->row_ptr[i]; p < Ain->row_ptr[i + 1]; ++p) put(inv[Ain->col[p]], Ain->val[p]);
  });
  sort_rows(A);
  clk.lap("permute");

  // symmetry check (informational: the method does not need it)
  s.symmetric = is_symmetric(A);
  check_grounded(A, s.symmetric);
  clk.lap("symmetry + grounding");

  std::vector<int32_t> rows_o(static_cast<size_t>(s.n_o)), rows_g(static_cast<size_t>(s.n_g));
  std::iota(rows_o.begin(), rows_o.end(), 0);
  std::iota(rows_g.begin(), rows_g.end(), s.n_o);
  std::vector<int32_t> map_o(static_cast<size_t>(n), -1), map_g(static_cast<size_t>(n), -1);
  for (int32_t i = 0; i < s.n_o; ++i) map_o[i] = i;
  for (int32_t i = 0; i < s.n_g; ++i) map_g[s.n_o + i] = i;
  s.Aoo = extract(A, rows_o, map_o, s.n_o);
  s.Aog = extract(A, rows_o, map_g, s.n_g);
  s.Ago = extract(A, rows_g, map_o, s.n_o);
  s.Agg = extract(A, rows_g, map_g, s.n_g);
  // eq. (7) divides by diag(A_GG) and the smoothers by the diagonals of S~
  // and A_GG; A itself may have zero diagonal entries (in the interface-flux
  // reading a point cell's row holds only interface terms)
  if (s.n_g > 0) check_diag(s.Agg, "A_GG");

  if (s.n_g > 0) {
    // S~ = A_OO - (A_OG diag(A_GG)^{-1}) A_GO   (eq. 7)
    const std::vector<double> d = diagonal(s.Agg);
    HCsr w = s.Aog;
    for (size_t p = 0; p < w.col.size(); ++p) w.val[p] = w.val[p] * (1.0 / d[w.col[p]]);
    s.S = subtract(s.Aoo, spgemm(w, s.Ago));
  } else {
    s.S = s.Aoo;
  }
  check_diag(s.S, "S~");
  clk.lap("blocks + S~");

  AmgParams prm;
  prm.theta = opt.strength_theta;
  prm.max_coarse = opt.max_coarse;
  prm.max_dense = opt.max_dense;
  prm.max_levels = opt.max_levels;
  std::vector<int32_t> lo, lg;
  if (label) {  // labels in [Omega; Gamma] order
    for (int32_t r = 0; r < s.n_o; ++r) lo.push_back(label[s.perm[r]]);
    for (int32_t r = s.n_o; r < n; ++r) lg.push_back(label[s.perm[r]]);
  }
  s.Ho = amg_setup(s.S, prm, label ? lo.data() : nullptr);
  if (s.n_g > 0) s.Hg = amg_setup(s.Agg, prm, label ? lg.data() : nullptr);
  s.A = std::move(A);
}

}  // namespace mdp
