// Device side of the solve phase: upload of host-built hierarchies (one
// system, or many concatenated block-diagonally), the V-cycle that defines
// Q_OO / Q_GG (Section 3.3), the preconditioner action of Algorithm 1 (M_L of
// eq. (8)) and right-preconditioned flexible GMRES (Section 3.2; zero
// initial guess and relative-residual stop, Section 4).
//
// Precision: the preconditioner runs in T (double, or float in mixed mode);
// the outer matrix, Krylov basis V, Hessenberg/Givens data and the coarsest
// dense inverses are always FP64.  Z (the preconditioned directions) is kept
// in T: A z_j is formed from the stored z_j, so FP32 storage is exact for the
// flexible method.
//
// Arnoldi: classical Gram-Schmidt whose reorthogonalisation of basis vector j
// is folded into step j+1 (one fused reduction pass and one update pass per
// step).  Reductions use fixed trees over fixed tiles, so results do not
// depend on scheduling.  Every (system, rhs) pair runs its own Krylov process
// with its own convergence test; whole-batch kernels (preconditioner, system
// matrix) stop once no pair needs them in the current cycle.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <string>
#include <mutex>
#include <tuple>
#include <type_traits>

#include "formats.hpp"
#include "kernels.hpp"
#include "ktimer.hpp"
#include "solver.hpp"

namespace mdp {

namespace {

// ---------------------------------------------------------------------------
// Upload helpers

template <typename T>
void upload_vec(DevMem &d, const std::vector<T> &h, hipStream_t s) {
  d.alloc(h.size() * sizeof(T));
  if (!h.empty()) MDP_HIP(hipMemcpyAsync(d.get(), h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

// Host staging buffers must outlive the asynchronous copies: they are kept
// here until the stream is synchronised.
struct Keep {
  std::vector<std::vector<int32_t>> i32;
  std::vector<std::vector<double>> f64;
  std::vector<std::vector<float>> f32;
  std::vector<std::vector<DenseDesc>> dd;
  std::vector<int32_t> &put(std::vector<int32_t> &&v) {
    i32.push_back(std::move(v));
    return i32.back();
  }
  std::vector<double> &put(std::vector<double> &&v) {
    f64.push_back(std::move(v));
    return f64.back();
  }
  std::vector<float> &put(std::vector<float> &&v) {
    f32.push_back(std::move(v));
    return f32.back();
  }
  std::vector<DenseDesc> &put(std::vector<DenseDesc> &&v) {
    dd.push_back(std::move(v));
    return dd.back();
  }
};

// Device formats of a sparse matrix, and the setup-time autotuner that picks
// one per matrix by timing the candidates on the device.
template <typename T>
void upload_csr_arrays(const HCsr &h, DCsr<T> &d, hipStream_t s, Keep &keep) {
  upload_vec(d.ptr, h.ptr, s);
  upload_vec(d.col, h.col, s);
  upload_vec(d.val, keep.put(std::vector<T>(h.val.begin(), h.val.end())), s);
}

template <typename T>
std::vector<T> as_type(const std::vector<double> &v) {
  return std::vector<T>(v.begin(), v.end());
}

template <typename T>
void upload_sell_arrays(const HCsr &h, DCsr<T> &d, const SliceStats &st, hipStream_t s, Keep &keep) {
  SellLayout L = sell_layout(h, st);
  d.nslices = L.nslices;
  upload_vec(d.ptr, keep.put(std::move(L.soff)), s);
  upload_vec(d.col, keep.put(std::move(L.col)), s);
  upload_vec(d.val, keep.put(as_type<T>(L.val)), s);
}

template <typename T>
void upload_dia_arrays(const HCsr &h, DCsr<T> &d, const std::vector<int32_t> &offs, hipStream_t s, Keep &keep) {
  DiaLayout L = dia_layout(h, offs);
  d.ndiag = static_cast<int32_t>(offs.size());
  upload_vec(d.ptr, keep.put(std::move(L.offs)), s);
  upload_vec(d.val, keep.put(as_type<T>(L.val)), s);
}

template <typename T>
void upload_hyb_arrays(const HCsr &h, DCsr<T> &d, const std::vector<int32_t> &offs, hipStream_t s, Keep &keep) {
  HybLayout L = hyb_layout(h, offs);
  d.ndiag = static_cast<int32_t>(offs.size());
  d.rem_nnz = static_cast<int64_t>(L.col.size());
  d.split = L.split;
  upload_vec(d.doff, keep.put(std::move(L.offs)), s);
  upload_vec(d.dval, keep.put(as_type<T>(L.dval)), s);
  upload_vec(d.ptr, keep.put(std::move(L.ptr)), s);
  upload_vec(d.col, keep.put(std::move(L.col)), s);
  upload_vec(d.val, keep.put(as_type<T>(L.val)), s);
}

// Autotuning is on while an AutotuneScope with on = true is alive on this
// thread (the setup paths open one from their options).
// The scope also owns the buffer that the timing reads to flush the caches,
// allocated on first use and freed with the scope.
thread_local bool t_autotune = false;
thread_local DevMem *t_flush = nullptr;

struct AutotuneScope {
  bool saved;
  DevMem *saved_flush;
  DevMem flush;
  explicit AutotuneScope(bool on) : saved(t_autotune), saved_flush(t_flush) {
    t_autotune = on;
    t_flush = &flush;
  }
  ~AutotuneScope() {
    t_autotune = saved;
    t_flush = saved_flush;
  }
};

// Choices already made in this process, by matrix signature, so that equal
// matrices get the same format (and so the same rounding) every time.
struct TuneKey {
  int vsize;
  int32_t nr, nc, maxlen;
  int64_t nnz, padded;
  bool operator<(const TuneKey &o) const {
    return std::tie(vsize, nr, nc, maxlen, nnz, padded) < std::tie(o.vsize, o.nr, o.nc, o.maxlen, o.nnz, o.padded);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, FormatChoice> g_tune;  // under g_tune_mu
std::string g_tune_path;                 // file that records the choices ("" = none), under g_tune_mu

// One choice per line: "vsize nr nc maxlen nnz padded  dia hyb sell scalar lpr batch".
void tune_record(const TuneKey &k, const FormatChoice &f) {
  if (g_tune_path.empty()) return;
  if (FILE *fp = std::fopen(g_tune_path.c_str(), "a")) {
    std::fprintf(fp, "%d %d %d %d %lld %lld  %d %d %d %d %d %d\n", k.vsize, k.nr, k.nc, k.maxlen,
                 static_cast<long long>(k.nnz), static_cast<long long>(k.padded), f.dia, f.hyb, f.sell, f.scalar,
                 f.lpr, f.batch);
    std::fclose(fp);
  }
}

// A restriction choice: "-vsize nr nc ncont nnz(Rf) nnz(R)  fused 0 0 0 4 4".
void tune_record_restriction(const TuneKey &k, bool fused) {
  if (g_tune_path.empty()) return;
  if (FILE *fp = std::fopen(g_tune_path.c_str(), "a")) {
    std::fprintf(fp, "%d %d %d %d %lld %lld  %d 0 0 0 4 %d\n", k.vsize, k.nr, k.nc, k.maxlen,
                 static_cast<long long>(k.nnz), static_cast<long long>(k.padded), fused ? 1 : 0, kCsrBatch);
    std::fclose(fp);
  }
}

bool valid_lpr(int l) { return l == 2 || l == 4 || l == 8 || l == 16 || l == 32 || l == 64 || l == kThreads; }

template <typename T>
FormatChoice autotune_format(const HCsr &h, const SliceStats &st, const std::vector<int32_t> &offs,
                             const std::vector<int32_t> &hoffs, hipStream_t s, Keep &keep, DCsr<T> &won,
                             bool &filled);

// Move the device arrays of a matrix, and the fields that describe them, from
// src into d (d's block and pair fields stay).
template <typename T>
void take_arrays(DCsr<T> &d, DCsr<T> &src) {
  d.ptr = std::move(src.ptr);
  d.col = std::move(src.col);
  d.val = std::move(src.val);
  d.doff = std::move(src.doff);
  d.dval = std::move(src.dval);
  d.ndiag = src.ndiag;
  d.rem_nnz = src.rem_nnz;
  d.split = src.split;
  d.nslices = src.nslices;
}

// Restriction of a level: true to keep the fused product R (I - A D^-1) b,
// false for the residual b - A D^-1 b and then R (see choose_fused).
std::map<TuneKey, int> g_rtune;  // under g_tune_mu
template <typename T>
bool choose_fused(const HCsr &rf, const DCsr<T> &Rf, const DCsr<T> &A, const DCsr<T> &R, hipStream_t s);

// Upload a host CSR in the device format that suits it.  With autotuning
// on, matrices of at least kTuneMinNnz entries are timed on the device in
// every candidate format and the fastest is kept.
constexpr int64_t kTuneMinNnz = 1 << 15;

template <typename T>
void upload_csr(const HCsr &h, DCsr<T> &d, hipStream_t s, Keep &keep) {
  d.nr = h.nr;
  d.nc = h.nc;
  d.nnz = h.nnz();
  const SliceStats st = slice_stats(h);
  const std::vector<int32_t> offs = h.nr > 0 ? dia_offsets(h) : std::vector<int32_t>{};
  const std::vector<int32_t> hoffs = offs.empty() ? hyb_offsets(h) : std::vector<int32_t>{};
  FormatChoice f = heuristic_format(h, st, !offs.empty(), !hoffs.empty());
  const auto t0 = std::chrono::steady_clock::now();
  // the autotuner hands over the arrays of the format it chose (filled), or
  // returns a recorded choice whose arrays are built here
  DCsr<T> won;
  bool filled = false;
  if (t_autotune && d.nnz >= kTuneMinNnz && h.nr > 0) f = autotune_format<T>(h, st, offs, hoffs, s, keep, won, filled);
  const auto t1 = std::chrono::steady_clock::now();
  d.dia = f.dia;
  d.hyb = f.hyb;
  d.sell = f.sell;
  d.scalar = f.scalar;
  d.lpr = f.lpr;
  d.batch = f.batch;
  if (filled)
    take_arrays(d, won);
  else if (f.dia)
    upload_dia_arrays(h, d, offs, s, keep);
  else if (f.hyb)
    upload_hyb_arrays(h, d, hoffs, s, keep);
  else if (f.sell)
    upload_sell_arrays(h, d, st, s, keep);
  else
    upload_csr_arrays(h, d, s, keep);
  if (std::getenv("MDP_SETUP_VERBOSE")) {
    const auto t2 = std::chrono::steady_clock::now();
    std::fprintf(stderr, "[mdp] upload n=%d nnz=%lld: tune %.3f s, upload %.3f s\n", h.nr,
                 static_cast<long long>(h.nnz()), std::chrono::duration<double>(t1 - t0).count(),
                 std::chrono::duration<double>(t2 - t1).count());
  }
}

using Piece = std::tuple<const HCsr *, int32_t, int32_t>;  // matrix, row offset, column offset

// Block-diagonal concatenation of pieces into an nr x nc matrix.
HCsr concat_blocks(int32_t nr, int32_t nc, const std::vector<Piece> &pieces) {
  std::vector<int32_t> rowlen(static_cast<size_t>(nr), 0);
  for (const auto &pc : pieces) {
    const HCsr &m = *std::get<0>(pc);
    const int32_t ro = std::get<1>(pc);
    for (int32_t i = 0; i < m.nr; ++i) rowlen[ro + i] = m.ptr[i + 1] - m.ptr[i];
  }
  HCsr out = HCsr::empty(nr, nc);
  for (int32_t i = 0; i < nr; ++i) out.ptr[i + 1] = out.ptr[i] + rowlen[i];
  out.col.resize(static_cast<size_t>(out.ptr[nr]));
  out.val.resize(static_cast<size_t>(out.ptr[nr]));
  for (const auto &pc : pieces) {
    const HCsr &m = *std::get<0>(pc);
    const int32_t ro = std::get<1>(pc), co = std::get<2>(pc);
    for (int32_t i = 0; i < m.nr; ++i) {
      int32_t q = out.ptr[ro + i];
      for (int32_t p = m.ptr[i]; p < m.ptr[i + 1]; ++p, ++q) {
        out.col[q] = m.col[p] + co;
        out.val[q] = m.val[p];
      }
    }
  }
  return out;
}

// Level orderings of a batch of hierarchies: at every level, systems that
// continue to the next level first, then dense-coarsest ones, then swept
// ones (each group in pair order).  off[l][p] = row offset of hierarchy p at
// level l (-1 if absent).
struct LevelPlan {
  std::vector<std::vector<int>> order;
  std::vector<std::vector<int64_t>> off;
  std::vector<int32_t> n, ncont, sw_off;
};

LevelPlan plan_levels(const std::vector<const HHier *> &hs, bool tails) {
  LevelPlan pl;
  size_t L = 0;
  for (const HHier *h : hs) L = std::max(L, h->depth(tails));
  pl.order.resize(L);
  pl.off.assign(L, std::vector<int64_t>(hs.size(), -1));
  pl.n.assign(L, 0);
  pl.ncont.assign(L, 0);
  pl.sw_off.assign(L, 0);
  for (size_t l = 0; l < L; ++l) {
    std::vector<int> cont, dense, sweep;
    for (size_t p = 0; p < hs.size(); ++p) {
      const HHier &h = *hs[p];
      if (h.depth(tails) <= l) continue;
      if (l + 1 < h.depth(tails))
        cont.push_back(static_cast<int>(p));
      else if (h.ends_dense(tails))
        dense.push_back(static_cast<int>(p));
      else
        sweep.push_back(static_cast<int>(p));
    }
    int64_t o = 0;
    auto place = [&](const std::vector<int> &v) {
      for (int p : v) {
        pl.off[l][p] = o;
        pl.order[l].push_back(p);
        o += hs[p]->lv[l].A.nr;
      }
    };
    place(cont);
    pl.ncont[l] = static_cast<int32_t>(o);
    place(dense);
    pl.sw_off[l] = static_cast<int32_t>(o);
    place(sweep);
    if (o > std::numeric_limits<int32_t>::max()) raise(MDP_EINVAL, "batch level exceeds int32 indexing");
    pl.n[l] = static_cast<int32_t>(o);
  }
  return pl;
}

// Distance between the two ping-pong buffers of a level's swept coarsest
// systems: their rows, or with kb blocks a whole level vector (block r of a
// buffer starts r * n further on).
template <typename T>
int64_t sweep_stride(const DLevel<T> &L, int kb) {
  return kb == 1 ? L.n - L.sw_off : static_cast<int64_t>(kb) * L.n;
}

// Upload a batch of hierarchies laid out by `pl`.  kb > 1: every level
// vector holds kb blocks of that layout (one per right-hand side) and the
// matrices, stored once, carry the blocks' strides.  pair_of (batches): the
// system of each hierarchy, for the row-to-system maps that gate stopped
// pairs' rows (pair of a row in block r = r * nsys + its system).
template <typename T>
void upload_hier(const std::vector<const HHier *> &hs, const LevelPlan &pl, DHier<T> &d, hipStream_t s, Keep &keep,
                 int pre, int post, bool gs, bool tails, const std::vector<int> *pair_of = nullptr, int kb = 1,
                 int nsys = 1) {
  const size_t L = pl.order.size();
  d.lv.clear();
  d.lv.resize(L);
  d.kb = kb;
  d.pre = pre;
  d.post = post;
  d.gs = gs;
  std::vector<double> cinv;
  for (size_t l = 0; l < L; ++l) {
    DLevel<T> &dl = d.lv[l];
    dl.n = pl.n[l];
    dl.ncont = pl.ncont[l];
    dl.sw_off = pl.sw_off[l];
    const size_t nfull = static_cast<size_t>(kb) * dl.n;
    std::vector<Piece> pa, pp, pr, pr_plain, psw;
    std::vector<T> dinv(nfull);
    std::vector<DenseDesc> desc;
    bool sw_all_diag = true;  // every swept system of this level has a diagonal matrix
    // the level restricts b with R (I - A D^-1) when every continuing system
    // has it and the pre-smoothing is the single l1-Jacobi sweep from zero D^-1 b
    dl.fused = dl.ncont > 0 && pre == 1 && !gs;
    for (int p : pl.order[l])
      if (l + 1 < hs[p]->depth(tails) && hs[p]->lv[l].Rf.nr == 0) dl.fused = false;
    for (int p : pl.order[l]) {
      const HHier &h = *hs[p];
      const HLevel &hl = h.lv[l];
      const int32_t o = static_cast<int32_t>(pl.off[l][p]);
      for (int32_t i = 0; i < hl.A.nr; ++i) dinv[o + i] = static_cast<T>(1.0 / hl.dl1[i]);
      if (l + 1 < h.depth(tails)) {
        const int32_t oc = static_cast<int32_t>(pl.off[l + 1][p]);
        pa.emplace_back(&hl.A, o, o);
        pp.emplace_back(&hl.P, o, oc);
        pr.emplace_back(dl.fused ? &hl.Rf : &hl.R, oc, o);
        pr_plain.emplace_back(&hl.R, oc, o);
      } else if (h.ends_dense(tails)) {
        for (int r = 0; r < kb; ++r)
          desc.push_back(DenseDesc{static_cast<int32_t>(r * dl.n + o), hl.A.nr, static_cast<int64_t>(cinv.size())});
        cinv.insert(cinv.end(), h.coarse_op(tails).begin(), h.coarse_op(tails).end());
        dl.max_dense_n = std::max(dl.max_dense_n, hl.A.nr);
      } else {
        psw.emplace_back(&hl.A, o - dl.sw_off, o - dl.sw_off);
        bool diag = true;
        for (int32_t i = 0; i < hl.A.nr && diag; ++i)
          diag = hl.A.ptr[i + 1] - hl.A.ptr[i] == 1 && hl.A.col[hl.A.ptr[i]] == i;
        sw_all_diag = sw_all_diag && diag;
      }
    }
    for (int r = 1; r < kb; ++r) std::copy(dinv.begin(), dinv.begin() + dl.n, dinv.begin() + r * dl.n);
    const HCsr Acat = concat_blocks(dl.ncont, dl.ncont, pa);
    upload_csr(Acat, dl.A, s, keep);
    if (gs && dl.ncont > 0) {
      // each continuing system coloured on its own; a colour of the level is
      // that colour's rows of every system, ascending
      std::vector<std::vector<int32_t>> by_colour;
      for (int p : pl.order[l]) {
        if (l + 1 >= hs[p]->depth(tails)) continue;
        const std::vector<int32_t> col = greedy_colours(hs[p]->lv[l].A);
        const int32_t o = static_cast<int32_t>(pl.off[l][p]);
        for (size_t i = 0; i < col.size(); ++i) {
          if (static_cast<size_t>(col[i]) >= by_colour.size()) by_colour.resize(static_cast<size_t>(col[i]) + 1);
          by_colour[col[i]].push_back(o + static_cast<int32_t>(i));
        }
      }
      std::vector<int32_t> rows;
      dl.gs_off.assign(1, 0);
      dl.gs_nnz.clear();
      for (auto &c : by_colour) {
        std::sort(c.begin(), c.end());
        int64_t nz = 0;
        for (int32_t r : c) nz += Acat.ptr[r + 1] - Acat.ptr[r];
        rows.insert(rows.end(), c.begin(), c.end());
        dl.gs_off.push_back(static_cast<int32_t>(rows.size()));
        dl.gs_nnz.push_back(nz);
      }
      dl.Ag.nr = dl.Ag.nc = dl.ncont;
      dl.Ag.nnz = Acat.nnz();
      upload_csr_arrays(Acat, dl.Ag, s, keep);
      upload_vec(dl.gs_rows, keep.put(std::move(rows)), s);
      std::vector<T> dg(nfull, T(0));
      for (int32_t i = 0; i < dl.ncont; ++i)
        for (int32_t q = Acat.ptr[i]; q < Acat.ptr[i + 1]; ++q)
          if (Acat.col[q] == i) dg[i] = static_cast<T>(1.0 / Acat.val[q]);
      for (int r = 1; r < kb; ++r) std::copy(dg.begin(), dg.begin() + dl.n, dg.begin() + r * dl.n);
      upload_vec(dl.dg, keep.put(std::move(dg)), s);
      const double avg = static_cast<double>(Acat.nnz()) / std::max<int32_t>(dl.ncont, 1);
      dl.gs_lpr = avg <= 12.0 ? 1 : (avg <= 96.0 ? 8 : 32);
    }
    if (l + 1 < L) {
      upload_csr(concat_blocks(dl.ncont, pl.n[l + 1], pp), dl.P, s, keep);
      const HCsr Rcat = concat_blocks(pl.n[l + 1], dl.ncont, pr);
      upload_csr(Rcat, dl.R, s, keep);
      if (dl.fused && t_autotune && Rcat.nnz() >= kTuneMinNnz) {
        // the fused product moves fewer bytes, but the residual's own format
        // (diagonals, say) can make the two products faster: time both
        DCsr<T> Rp;
        upload_csr(concat_blocks(pl.n[l + 1], dl.ncont, pr_plain), Rp, s, keep);
        if (!choose_fused<T>(Rcat, dl.R, dl.A, Rp, s)) {
          dl.R = std::move(Rp);
          dl.fused = false;
        }
      }
    }
    upload_csr(concat_blocks(dl.n - dl.sw_off, dl.n - dl.sw_off, psw), dl.Asw, s, keep);
    dl.sw_diag = dl.n > dl.sw_off && sw_all_diag;
    dl.ndense = static_cast<int32_t>(desc.size());
    upload_vec(dl.dense, keep.put(std::move(desc)), s);
    upload_vec(dl.dinv, keep.put(std::move(dinv)), s);
    const size_t nb = std::max<size_t>(nfull, 1) * sizeof(T);
    dl.x.alloc(nb);
    dl.b.alloc(nb);
    dl.t.alloc(nb);
    if (!dl.fused || post > 1 || gs) dl.r.alloc(nb);  // residual; sweep ping-pong
    if (dl.n > dl.sw_off) dl.pp.alloc(2 * sweep_stride(dl, kb) * sizeof(T));
    // block strides: x of A, P, R and Asw lives on levels l, l + 1, l and l;
    // their b / dinv / y on levels l, l, l + 1 and l
    const int64_t nl = dl.n, nc = l + 1 < L ? pl.n[l + 1] : 0;
    auto blocks = [&](DCsr<T> &M, int64_t xs, int64_t ys) {
      M.kb = kb;
      M.bxs = xs;
      M.bys = ys;
      M.nsys = nsys;
    };
    blocks(dl.A, nl, nl);
    blocks(dl.P, nc, nl);
    blocks(dl.R, nl, nc);
    blocks(dl.Asw, nl, nl);
  }
  upload_vec(d.cinv, keep.put(std::move(cinv)), s);
  const size_t n0 = static_cast<size_t>(std::max<int64_t>(d.nfull(), 1)) * sizeof(T);
  d.tmp_res.alloc(n0);
  d.tmp_dz.alloc(n0);
  if (pair_of) {
    // per level, the system owning each row (hierarchy p belongs to pair_of[p])
    d.rowpair.clear();
    d.rowpair.resize(L);
    for (size_t l = 0; l < L; ++l) {
      std::vector<int32_t> m(static_cast<size_t>(pl.n[l]), -1);
      for (int p : pl.order[l]) {
        const int64_t o = pl.off[l][p];
        std::fill(m.begin() + o, m.begin() + o + hs[p]->lv[l].A.nr, (*pair_of)[p]);
      }
      if (std::find(m.begin(), m.end(), -1) != m.end()) raise(MDP_EINVAL, "batch level row without a pair");
      upload_vec(d.rowpair[l], keep.put(std::move(m)), s);
    }
    for (size_t l = 0; l < L; ++l) {
      DLevel<T> &dl = d.lv[l];
      const int *m = dptr<const int>(d.rowpair[l]);
      dl.A.rowpair = m;  // rows: the continuing systems' rows of level l
      dl.P.rowpair = m;
      if (l + 1 < L) dl.R.rowpair = dptr<const int>(d.rowpair[l + 1]);  // rows: level l + 1
      dl.Asw.rowpair = m + dl.sw_off;
    }
  }
}

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(b, 8192)));
}

// ---------------------------------------------------------------------------
// Sparse products

// Launch gating.  `all` (a device flag) retires a whole launch once every
// pair has stopped applying the preconditioner; with `st` (batched solves)
// the sparse products also skip the rows of pairs that have stopped, through
// each matrix's row-to-pair map.
struct Gate {
  const int *all = nullptr;
  const GmresState *st = nullptr;
};

// Algorithmic bytes of one sparse product: matrix values, column indices and
// row pointers once, each vector entry read or written once.
template <int MODE, typename TA, typename TX, typename TY>
double spmv_bytes(const DCsr<TA> &A) {
  // every stored value and index once: diagonal storage keeps ndiag values
  // per row (zeros included) and no indices
  double b = A.dia ? static_cast<double>(sizeof(TA)) * A.ndiag * A.nr + 4.0 * A.ndiag
                   : (sizeof(TA) + 4.0) * A.nnz + 4.0 * (A.nr + 1.0);
  if (A.hyb)  // diagonals (zeros included), then the remainder's entries and row pointers
    b = static_cast<double>(sizeof(TA)) * A.ndiag * A.nr + 4.0 * A.ndiag + (sizeof(TA) + 4.0) * A.rem_nnz +
        4.0 * (A.nr + 1.0);
  const double sx = sizeof(TX) * A.kb, sy = sizeof(TY) * A.kb;  // vectors once per block
  if (MODE == kPlain) b += sx * A.nc + sy * A.nr;
  if (MODE == kResid) b += sx * A.nc + 2 * sy * A.nr;
  if (MODE == kSmooth) b += sx * A.nc + 3 * sy * A.nr;      // x, b, dinv, y
  if (MODE == kAccum) b += sx * A.nc + 2 * sy * A.nr;
  if (MODE == kPlainScale) b += sx * A.nc + 3 * sy * A.nr;  // x; dinv, y, y2
  if (MODE == kResidScale) b += sx * A.nc + 4 * sy * A.nr;  // x; b, dinv, y, y2
  return b;
}

template <int LPR, int BATCH, int KB, int MODE, typename TA, typename TX, typename TY>
void spmv_launch(const DCsr<TA> &A, const TX *x, const TY *b, const TY *dinv, TY *y, TY *y2, Gate gate,
                 hipStream_t s, int kind) {
  const int64_t rows_per_blk = kThreads / LPR;
  const int blocks = static_cast<int>((A.nr + rows_per_blk - 1) / rows_per_blk);
  const Blocks bk{A.bxs, A.bys, A.nsys};
  timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
    hipLaunchKernelGGL((spmv_kernel<LPR, BATCH, KB, MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr,
                       A.p(), A.c(), A.v(), x, b, dinv, y, y2, gate.all, gate.st ? A.rp() : nullptr, gate.st, bk);
  });
}

template <int BATCH, int KB, int MODE, typename TA, typename TX, typename TY>
void spmv_row_block_launch(const DCsr<TA> &A, const TX *x, const TY *b, const TY *dinv, TY *y, TY *y2, Gate gate,
                           hipStream_t s, int kind) {
  const Blocks bk{A.bxs, A.bys, A.nsys};
  timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
    hipLaunchKernelGGL((spmv_row_block_kernel<BATCH, KB, MODE, TA, TX, TY>), dim3(A.nr), dim3(kThreads), 0, s, A.nr,
                       A.p(), A.c(), A.v(), x, b, dinv, y, y2, gate.all, gate.st ? A.rp() : nullptr, gate.st, bk);
  });
}

template <int KB, int MODE, typename TA, typename TX, typename TY>
void spmv_kb(const DCsr<TA> &A, const TX *x, const TY *b, const TY *dinv, TY *y, TY *y2, Gate gate,
             hipStream_t s, int kind) {
  const Blocks bk{A.bxs, A.bys, A.nsys};
  const int *rp = gate.st ? A.rp() : nullptr;
  if (A.dia) {
    const int blocks = (A.nr + kThreads - 1) / kThreads;
    timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
      hipLaunchKernelGGL((dia_kernel<KB, MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr, A.nc,
                         A.ndiag, A.p(), A.v(), x, b, dinv, y, y2, gate.all, rp, gate.st, bk);
    });
    return;
  }
  if (A.hyb) {
    const int blocks = hyb_blocks(A.nr, A.split);
    timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
      hipLaunchKernelGGL((hyb_kernel<KB, MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr, A.nc,
                         A.split, A.ndiag, dptr<const int>(A.doff), dptr<const TA>(A.dval), A.p(), A.c(), A.v(), x,
                         b, dinv, y, y2, gate.all, rp, gate.st, bk);
    });
    return;
  }
  if (A.sell) {
    const int blocks = (A.nslices + (kThreads / 64) - 1) / (kThreads / 64);
    timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
      hipLaunchKernelGGL((sell_kernel<KB, MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr, A.nslices,
                         A.p(), A.c(), A.v(), x, b, dinv, y, y2, gate.all, rp, gate.st, bk);
    });
    return;
  }
  if (A.scalar) {
    const int blocks = (A.nr + kThreads - 1) / kThreads;
    timed_launch(kind, s, spmv_bytes<MODE, TA, TX, TY>(A), [&] {
      hipLaunchKernelGGL((csr_scalar_kernel<KB, MODE, TA, TX, TY>), dim3(blocks), dim3(kThreads), 0, s, A.nr,
                         A.p(), A.c(), A.v(), x, b, dinv, y, y2, gate.all, rp, gate.st, bk);
    });
    return;
  }
  const bool b8 = A.batch == 8;
  switch (A.lpr) {
#define MDP_LPR_CASE(L)                                                         \
  case L:                                                                       \
    if (b8)                                                                     \
      spmv_launch<L, 8, KB, MODE>(A, x, b, dinv, y, y2, gate, s, kind);         \
    else                                                                        \
      spmv_launch<L, kCsrBatch, KB, MODE>(A, x, b, dinv, y, y2, gate, s, kind); \
    break;
    MDP_LPR_CASE(2)
    MDP_LPR_CASE(4)
    MDP_LPR_CASE(8)
    MDP_LPR_CASE(16)
    MDP_LPR_CASE(32)
    MDP_LPR_CASE(64)
#undef MDP_LPR_CASE
    case kThreads:  // one workgroup per row
      if (b8)
        spmv_row_block_launch<8, KB, MODE>(A, x, b, dinv, y, y2, gate, s, kind);
      else
        spmv_row_block_launch<kCsrBatch, KB, MODE>(A, x, b, dinv, y, y2, gate, s, kind);
      break;
    default: raise(MDP_EINVAL, "unsupported lanes per row");
  }
}

// y = op(A) x over A.kb vector blocks (one matrix read for all of them).
template <int MODE, typename TA, typename TX, typename TY>
void spmv(const DCsr<TA> &A, const TX *x, const TY *b, const TY *dinv, TY *y, TY *y2, Gate gate,
          hipStream_t s, int kind = kKcOther) {
  if (A.nr == 0) return;
  if (A.kb == kMultiRhs)
    spmv_kb<kMultiRhs, MODE>(A, x, b, dinv, y, y2, gate, s, kind);
  else if (A.kb == 1)
    spmv_kb<1, MODE>(A, x, b, dinv, y, y2, gate, s, kind);
  else
    raise(MDP_EINVAL, "unsupported number of vector blocks");
}

template <typename T>
const T *cnull() {
  return static_cast<const T *>(nullptr);
}
template <typename T>
T *mnull() {
  return static_cast<T *>(nullptr);
}

// Time every candidate format of one matrix (residual products, after two
// untimed ones) and return the fastest.  Candidates: CSR with 2..64 lanes per
// row or a whole workgroup per row, and 4 entries in flight per lane (also 8
// when a lane averages more than 4), CSR with one thread per row, sliced ELL when its padding stays within
// 2x, and the diagonal layouts when the matrix has them.  Each of kTuneColdReps
// timed products starts with cold caches, as inside a solve, where a V-cycle
// streams far more than the caches hold between two products with one matrix:
// a read of kFlushBytes (more than the 256 MB Infinity Cache and the L2s
// together) precedes it.  Without the flush buffer (out of memory) kTuneReps
// products run back to back.
constexpr int kTuneReps = 10;
constexpr int kTuneColdReps = 4;
constexpr size_t kFlushBytes = size_t(384) << 20;

void flush_caches(const DevMem &buf, hipStream_t s) {
  const int64_t n = static_cast<int64_t>(buf.bytes() / 16);
  hipLaunchKernelGGL(cache_flush_kernel, dim3(2048), dim3(kThreads), 0, s, dptr<const double2>(buf), n, 1.0,
                     dptr<double>(buf));
  MDP_HIP(hipGetLastError());
}

template <typename T>
FormatChoice autotune_format(const HCsr &h, const SliceStats &st, const std::vector<int32_t> &offs,
                             const std::vector<int32_t> &hoffs, hipStream_t s, Keep &keep, DCsr<T> &won,
                             bool &filled) {
  filled = false;
  const TuneKey key{static_cast<int>(sizeof(T)), h.nr, h.nc, st.maxlen, h.nnz(), st.padded};
  {
    // a recorded choice is used when this matrix has that layout
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      const FormatChoice &f = it->second;
      if ((!f.dia || !offs.empty()) && (!f.hyb || !hoffs.empty()) && (!f.sell || sell_possible(st, h.nnz(), 2.0)))
        return f;
      g_tune.erase(it);
    }
  }
  DCsr<T> csr;
  csr.nr = h.nr;
  csr.nc = h.nc;
  csr.nnz = h.nnz();
  upload_csr_arrays(h, csr, s, keep);
  DCsr<T> sell;
  const bool has_sell = sell_possible(st, h.nnz(), 2.0);
  if (has_sell) {
    sell.nr = h.nr;
    sell.nc = h.nc;
    sell.nnz = h.nnz();
    sell.sell = true;
    upload_sell_arrays(h, sell, st, s, keep);
  }
  DCsr<T> dia;
  if (!offs.empty()) {
    dia.nr = h.nr;
    dia.nc = h.nc;
    dia.nnz = h.nnz();
    dia.dia = true;
    upload_dia_arrays(h, dia, offs, s, keep);
  }
  DCsr<T> hyb;
  if (!hoffs.empty()) {
    hyb.nr = h.nr;
    hyb.nc = h.nc;
    hyb.nnz = h.nnz();
    hyb.hyb = true;
    upload_hyb_arrays(h, hyb, hoffs, s, keep);
  }
  DevMem xv(sizeof(T) * std::max<int32_t>(h.nc, 1)), bv(sizeof(T) * h.nr), yv(sizeof(T) * h.nr);
  MDP_HIP(hipMemsetAsync(xv.get(), 0, xv.bytes(), s));
  MDP_HIP(hipMemsetAsync(bv.get(), 0, bv.bytes(), s));
  const T *x = dptr<const T>(xv), *b = dptr<const T>(bv);
  T *y = dptr<T>(yv);
  DevMem *flush = t_flush;
  if (flush && !flush->get()) {
    try {
      flush->alloc(kFlushBytes);
      MDP_HIP(hipMemsetAsync(flush->get(), 0, kFlushBytes, s));
    } catch (const Error &e) {
      if (e.code != MDP_ENOMEM) throw;
      (void)hipGetLastError();
    }
  }
  const bool cold = flush && flush->get();
  const int reps = cold ? kTuneColdReps : kTuneReps;
  Events ev(2 * reps);
  // cold: one event pair around each product; warm: one pair around them all
  auto time_one = [&](const DCsr<T> &d) {
    for (int i = 0; i < 2; ++i) spmv<kResid>(d, x, b, cnull<T>(), y, mnull<T>(), Gate{}, s);
    for (int i = 0; i < reps; ++i) {
      if (cold) flush_caches(*flush, s);
      if (cold || i == 0) MDP_HIP(hipEventRecord(ev[2 * i], s));
      spmv<kResid>(d, x, b, cnull<T>(), y, mnull<T>(), Gate{}, s);
      if (cold || i == reps - 1) MDP_HIP(hipEventRecord(ev[2 * i + 1], s));
    }
    MDP_HIP(hipEventSynchronize(ev[2 * reps - 1]));
    float total = 0.f;
    for (int i = 0; i < (cold ? reps : 1); ++i) {
      float ms = 0.f;
      MDP_HIP(hipEventElapsedTime(&ms, ev[2 * i], ev[cold ? 2 * i + 1 : 2 * reps - 1]));
      total += ms;
    }
    return total / reps;
  };
  FormatChoice best = heuristic_format(h, st, !offs.empty(), !hoffs.empty());
  float tbest = std::numeric_limits<float>::max();
  // CSR-vector shapes whose lanes are neither mostly idle (more lanes than
  // twice the average row) nor too few (a row needing more than four steps;
  // the 64-lane shape is always tried, whatever the row length); a workgroup
  // per row when rows average at least 128 entries
  const double avg = static_cast<double>(h.nnz()) / h.nr;
  std::vector<FormatChoice> cand;
  for (int l : {2, 4, 8, 16, 32, 64, kThreads})
    for (int bt : {kCsrBatch, 8})
      if (l <= std::max(2.0, 2.0 * avg) && (4.0 * l * bt >= avg || l == 64) &&
          (bt == kCsrBatch || l * kCsrBatch < avg))
        cand.push_back(FormatChoice{false, false, l, bt});
  cand.push_back(FormatChoice{false, true, 4, kCsrBatch});
  for (const FormatChoice &c : cand) {
    csr.scalar = c.scalar;
    csr.lpr = c.lpr;
    csr.batch = c.batch;
    const float t = time_one(csr);
    if (t < tbest) tbest = t, best = c;
  }
  if (has_sell) {
    const float t = time_one(sell);
    if (t < tbest) tbest = t, best = FormatChoice{true, false, 8, kCsrBatch};
  }
  if (!offs.empty()) {
    const float t = time_one(dia);
    if (t < tbest) tbest = t, best = FormatChoice{false, false, 8, kCsrBatch, true};
  }
  if (!hoffs.empty()) {
    const float t = time_one(hyb);
    if (t < tbest) tbest = t, best = FormatChoice{false, false, 8, kCsrBatch, false, true};
  }
  MDP_HIP(hipStreamSynchronize(s));
  if (std::getenv("MDP_SETUP_VERBOSE"))
    std::fprintf(stderr, "[mdp] autotune %s n=%d nnz=%lld: %s lpr=%d batch=%d (%.2f us)\n",
                 sizeof(T) == 8 ? "f64" : "f32", h.nr, static_cast<long long>(h.nnz()),
                 best.dia ? "dia" : best.hyb ? "dia+csr" : best.sell ? "sell" : best.scalar ? "scalar" : "csr-vector",
                 best.lpr, best.batch, 1e3 * tbest);
  // a choice recorded meanwhile by another thread for the same signature
  // wins, so that equal matrices get one format
  FormatChoice chosen = best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto ins = g_tune.emplace(key, best);
    if (ins.second) {
      tune_record(key, best);
    } else {
      const FormatChoice &f = ins.first->second;
      if ((!f.dia || !offs.empty()) && (!f.hyb || !hoffs.empty()) && (!f.sell || has_sell)) chosen = f;
    }
  }
  take_arrays(won, chosen.dia ? dia : chosen.hyb ? hyb : chosen.sell ? sell : csr);
  filled = true;
  return chosen;
}

// Time the two ways of restricting b on one level, each from cold caches as
// in autotune_format: the fused product Rf b, and the residual b - A D^-1 b
// followed by R of it.  A recorded choice is used without timing.
template <typename T>
bool choose_fused(const HCsr &rf, const DCsr<T> &Rf, const DCsr<T> &A, const DCsr<T> &R, hipStream_t s) {
  const TuneKey key{-static_cast<int>(sizeof(T)), rf.nr, rf.nc, A.nr, rf.nnz(), R.nnz};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_rtune.find(key);
    if (it != g_rtune.end()) return it->second != 0;
  }
  const int64_t nf = std::max<int32_t>(A.nr, 1), nc = std::max<int32_t>(Rf.nr, 1);
  DevMem bv(sizeof(T) * nf), tv(sizeof(T) * nf), rv(sizeof(T) * nf), dv(sizeof(T) * nf);
  DevMem yc(sizeof(T) * nc), y2c(sizeof(T) * nc), dc(sizeof(T) * nc);
  for (DevMem *d : {&bv, &tv, &rv, &dv, &yc, &y2c, &dc}) MDP_HIP(hipMemsetAsync(d->get(), 0, d->bytes(), s));
  DevMem *flush = t_flush;
  if (flush && !flush->get()) {
    try {
      flush->alloc(kFlushBytes);
      MDP_HIP(hipMemsetAsync(flush->get(), 0, kFlushBytes, s));
    } catch (const Error &e) {
      if (e.code != MDP_ENOMEM) throw;
      (void)hipGetLastError();
    }
  }
  const bool cold = flush && flush->get();
  const int reps = cold ? kTuneColdReps : kTuneReps;
  Events ev(2);
  auto fused = [&] {
    spmv<kPlainScale>(Rf, dptr<const T>(bv), cnull<T>(), dptr<const T>(dc), dptr<T>(yc), dptr<T>(y2c), Gate{}, s);
  };
  auto unfused = [&] {
    spmv<kResid>(A, dptr<const T>(tv), dptr<const T>(bv), dptr<const T>(dv), dptr<T>(rv), mnull<T>(), Gate{}, s);
    spmv<kPlainScale>(R, dptr<const T>(rv), cnull<T>(), dptr<const T>(dc), dptr<T>(yc), dptr<T>(y2c), Gate{}, s);
  };
  auto time_route = [&](auto &&route) {
    route();
    route();
    float total = 0.f;
    for (int i = 0; i < reps; ++i) {
      if (cold) flush_caches(*flush, s);
      MDP_HIP(hipEventRecord(ev[0], s));
      route();
      MDP_HIP(hipEventRecord(ev[1], s));
      MDP_HIP(hipEventSynchronize(ev[1]));
      float ms = 0.f;
      MDP_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
      total += ms;
    }
    return total / reps;
  };
  const float tf = time_route(fused), tu = time_route(unfused);
  const bool keep_fused = tf <= tu;
  MDP_HIP(hipStreamSynchronize(s));
  if (std::getenv("MDP_SETUP_VERBOSE"))
    std::fprintf(stderr, "[mdp] restriction %s rows=%d: fused %.2f us, residual + R %.2f us -> %s\n",
                 sizeof(T) == 8 ? "f64" : "f32", rf.nr, 1e3 * tf, 1e3 * tu, keep_fused ? "fused" : "residual + R");
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (g_rtune.emplace(key, keep_fused ? 1 : 0).second) tune_record_restriction(key, keep_fused);
  return keep_fused;
}

}  // namespace

void set_tune_file(const char *path) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune_path.clear();
  if (!path) return;
  if (FILE *fp = std::fopen(path, "r")) {
    // earlier choices take precedence over timing; malformed lines are skipped
    char line[256];
    while (std::fgets(line, sizeof line, fp)) {
      TuneKey k{};
      long long nnz = 0, padded = 0;
      int dia = 0, hyb = 0, sell = 0, scalar = 0, lpr = 0, batch = 0;
      if (std::sscanf(line, "%d %d %d %d %lld %lld %d %d %d %d %d %d", &k.vsize, &k.nr, &k.nc, &k.maxlen, &nnz,
                      &padded, &dia, &hyb, &sell, &scalar, &lpr, &batch) != 12)
        continue;
      if ((k.vsize == -4 || k.vsize == -8) && (dia == 0 || dia == 1) && hyb + sell + scalar == 0) {
        k.nnz = nnz;
        k.padded = padded;
        g_rtune[k] = dia;
        continue;
      }
      if ((k.vsize != 4 && k.vsize != 8) || dia + hyb + sell + scalar > 1 || !valid_lpr(lpr) ||
          (batch != kCsrBatch && batch != 8))
        continue;
      k.nnz = nnz;
      k.padded = padded;
      g_tune[k] = FormatChoice{sell != 0, scalar != 0, lpr, batch, dia != 0, hyb != 0};
    }
    std::fclose(fp);
  } else if (FILE *fp2 = std::fopen(path, "a")) {
    std::fclose(fp2);
  } else {
    raise(MDP_EINVAL, std::string("cannot open the tuning file ") + path);
  }
  g_tune_path = path;
}

namespace {

// ---------------------------------------------------------------------------
// V-cycle (Section 3.3): l1-Jacobi pre-smoothing from zero, residual,
// restriction, coarse correction, prolongation, l1-Jacobi post-smoothing.
//
// The finest level's scratch `t` must hold the first smoothing iterate
// x0 = D^-1 b on entry; the kernels that produce b also write x0
// (restriction, the fracture-residual update, the input cast), so the
// smoother's residual needs one gather per nonzero.

template <typename T>
void start_smoother(DHier<T> &H, const T *b, Gate gate, hipStream_t s) {
  const int64_t n = H.nfull();
  if (n == 0 || H.dense_only()) return;
  timed_launch(kKcVcycleOther, s, 3.0 * sizeof(T) * n, [&] {
    hipLaunchKernelGGL(diag_scale_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, static_cast<int>(n), b,
                       dptr<const T>(H.lv[0].dinv), dptr<T>(H.lv[0].t), gate.all);
  });
}

// Systems whose coarsest level is l: dense inverses, or four l1-Jacobi sweeps
// from zero (the first, D^-1 b, is already in t).
template <typename T>
void coarse_solve(DHier<T> &H, DLevel<T> &L, const T *b, T *x, Gate gate, hipStream_t s) {
  if (L.ndense > 0) {
    const dim3 grid((L.max_dense_n + (kThreads / 64) - 1) / (kThreads / 64), L.ndense);
    timed_launch(kKcVcycleOther, s, 0.0, [&] {
      hipLaunchKernelGGL(dense_gemv_batched_kernel<T>, grid, dim3(kThreads), 0, s, dptr<const DenseDesc>(L.dense),
                         dptr<const double>(H.cinv), b, x, gate.all);
    });
  }
  const int nsw = L.n - L.sw_off;
  if (nsw > 0 && L.sw_diag) {
    // diagonal systems (A_GG of the interface-flux reading): the first
    // l1-Jacobi iterate D^-1 b, already in t, is their solution, and further
    // sweeps would only add rounding
    const int o = L.sw_off;
    for (int r = 0; r < H.kb; ++r) {
      const int64_t off = static_cast<int64_t>(r) * L.n + o;
      timed_launch(kKcVcycleOther, s, 2.0 * sizeof(T) * nsw, [&] {
        hipLaunchKernelGGL((scale_copy_kernel<T, T>), dim3(grid_for(nsw)), dim3(kThreads), 0, s,
                           static_cast<int64_t>(nsw), dptr<const T>(L.t) + off, static_cast<const double *>(nullptr),
                           x + off, gate.all);
      });
    }
  } else if (nsw > 0) {
    const int o = L.sw_off;
    T *pa = dptr<T>(L.pp), *pb = pa + sweep_stride(L, H.kb);
    const T *t = dptr<const T>(L.t) + o;
    const T *dinv = dptr<const T>(L.dinv) + o;
    const int kc = kKcVcycleOther;
    spmv<kSmooth>(L.Asw, t, b + o, dinv, pa, mnull<T>(), gate, s, kc);
    spmv<kSmooth>(L.Asw, static_cast<const T *>(pa), b + o, dinv, pb, mnull<T>(), gate, s, kc);
    spmv<kSmooth>(L.Asw, static_cast<const T *>(pb), b + o, dinv, x + o, mnull<T>(), gate, s, kc);
  }
}

// One multicolour Gauss-Seidel sweep on level L (forward: colours ascending).
template <int LPR, int KB, typename T>
void gs_launch(DLevel<T> &L, int c, const T *b, T *x, Gate gate, hipStream_t s, int kind) {
  const int nrows = L.gs_off[c + 1] - L.gs_off[c];
  if (nrows == 0) return;
  const int64_t threads = static_cast<int64_t>(nrows) * LPR;
  const int blocks = static_cast<int>((threads + kThreads - 1) / kThreads);
  const Blocks bk{L.A.bxs, L.A.bys, L.A.nsys};
  const double bytes = (sizeof(T) + 4.0) * L.gs_nnz[c] + 12.0 * nrows + 3.0 * sizeof(T) * KB * nrows;
  timed_launch(kind, s, bytes, [&] {
    hipLaunchKernelGGL((gs_colour_kernel<LPR, KB, T, T>), dim3(blocks), dim3(kThreads), 0, s, nrows,
                       dptr<const int>(L.gs_rows) + L.gs_off[c], L.Ag.p(), L.Ag.c(), L.Ag.v(),
                       dptr<const T>(L.dg), b, x, gate.all, bk);
  });
}

template <int KB, typename T>
void gs_sweep_kb(DLevel<T> &L, bool forward, const T *b, T *x, Gate gate, hipStream_t s, int kind) {
  const int nc = static_cast<int>(L.gs_off.size()) - 1;
  for (int k = 0; k < nc; ++k) {
    const int c = forward ? k : nc - 1 - k;
    if (L.gs_lpr == 1)
      gs_launch<1, KB>(L, c, b, x, gate, s, kind);
    else if (L.gs_lpr == 8)
      gs_launch<8, KB>(L, c, b, x, gate, s, kind);
    else
      gs_launch<32, KB>(L, c, b, x, gate, s, kind);
  }
}

template <typename T>
void gs_sweep(DHier<T> &H, DLevel<T> &L, bool forward, const T *b, T *x, Gate gate, hipStream_t s, int kind) {
  if (H.kb == kMultiRhs)
    gs_sweep_kb<kMultiRhs>(L, forward, b, x, gate, s, kind);
  else
    gs_sweep_kb<1>(L, forward, b, x, gate, s, kind);
}

template <typename T>
void vcycle(DHier<T> &H, size_t l, const T *b, T *x, Gate gate, hipStream_t s) {
  DLevel<T> &L = H.lv[l];
  if (L.ncont > 0 && H.gs) {
    // Gauss-Seidel: forward sweeps from zero in place on x, the residual and
    // its restriction, the coarse correction, backward sweeps
    DLevel<T> &C = H.lv[l + 1];
    const bool fine = H.is_omega && l == 0;
    const int ks = fine ? kKcFineSmooth : kKcVcycleOther;
    const int kr = fine ? kKcFineResid : kKcVcycleOther;
    const int ko = kKcVcycleOther;
    const int64_t nf = static_cast<int64_t>(H.kb) * L.n;
    hipLaunchKernelGGL(zero_kernel<T>, dim3(grid_for(nf)), dim3(kThreads), 0, s, static_cast<int>(nf), x, gate.all);
    for (int k = 0; k < H.pre; ++k) gs_sweep(H, L, true, b, x, gate, s, ks);
    spmv<kResid>(L.A, static_cast<const T *>(x), b, dptr<const T>(L.dinv), dptr<T>(L.r), mnull<T>(), gate, s, kr);
    spmv<kPlainScale>(L.R, dptr<const T>(L.r), cnull<T>(), dptr<const T>(C.dinv), dptr<T>(C.b), dptr<T>(C.t), gate, s,
                      ko);
    vcycle(H, l + 1, dptr<const T>(C.b), dptr<T>(C.x), gate, s);
    spmv<kAccum>(L.P, dptr<const T>(C.x), cnull<T>(), cnull<T>(), x, mnull<T>(), gate, s, ko);  // x += P x_c
    for (int k = 0; k < H.post; ++k) gs_sweep(H, L, false, b, x, gate, s, ks);
  } else if (L.ncont > 0) {
    DLevel<T> &C = H.lv[l + 1];
    T *t = dptr<T>(L.t), *r = dptr<T>(L.r);
    const T *dinv = dptr<const T>(L.dinv);
    const bool fine = H.is_omega && l == 0;
    const int ks = fine ? kKcFineSmooth : kKcVcycleOther;
    const int kr = fine ? kKcFineResid : kKcVcycleOther;
    const int ko = kKcVcycleOther;
    // pre-smoothing from zero: the first iterate is t = D^-1 b; further
    // sweeps alternate between t and r
    T *cur = t;
    for (int k = 1; k < H.pre; ++k) {
      T *nxt = cur == t ? r : t;
      spmv<kSmooth>(L.A, static_cast<const T *>(cur), b, dinv, nxt, mnull<T>(), gate, s, ks);
      cur = nxt;
    }
    // residual b - A cur, in the buffer of t and r that cur does not hold
    T *res = cur == t ? r : t;
    if (!L.fused) spmv<kResid>(L.A, static_cast<const T *>(cur), b, dinv, res, mnull<T>(), gate, s, kr);
    // b_c = R res (fused: R (I - A D^-1) b, the same vector) and the coarse
    // level's first iterate t_c = D_c^-1 b_c
    spmv<kPlainScale>(L.R, L.fused ? b : static_cast<const T *>(res), cnull<T>(), dptr<const T>(C.dinv),
                      dptr<T>(C.b), dptr<T>(C.t), gate, s, L.fused && fine ? kr : ko);
    vcycle(H, l + 1, dptr<const T>(C.b), dptr<T>(C.x), gate, s);
    spmv<kAccum>(L.P, dptr<const T>(C.x), cnull<T>(), cnull<T>(), cur, mnull<T>(), gate, s, ko);  // cur += P x_c
    // post-smoothing: the last sweep writes x, earlier ones alternate
    // between t and r
    for (int k = 0; k < H.post; ++k) {
      T *nxt = k + 1 == H.post ? x : (cur == t ? r : t);
      spmv<kSmooth>(L.A, static_cast<const T *>(cur), b, dinv, nxt, mnull<T>(), gate, s, ks);
      cur = nxt;
    }
  }
  if (L.ncont < L.n) coarse_solve(H, L, b, x, gate, s);
}

// Q = `cycles` V-cycles as a stationary iteration from zero (lv[0].t = D^-1 r on entry).
template <typename T>
void apply_q(DHier<T> &H, int cycles, const T *r, T *z, Gate gate, hipStream_t s) {
  {
    const Range range("V-cycle");
    vcycle(H, 0, r, z, gate, s);
  }
  const int64_t n = H.nfull();
  DLevel<T> &L0 = H.lv[0];
  for (int c = 1; c < cycles; ++c) {
    // residual r - A z and its first smoothing iterate, for the continuing
    // and the swept systems; dense-solved systems are exact already, so their
    // residual is zero
    spmv<kResidScale>(L0.A, static_cast<const T *>(z), r, dptr<const T>(L0.dinv), dptr<T>(H.tmp_res), dptr<T>(L0.t),
                      gate, s, kKcVcycleOther);
    const int o = L0.sw_off;
    if (L0.n > o)
      spmv<kResidScale>(L0.Asw, static_cast<const T *>(z) + o, r + o, dptr<const T>(L0.dinv) + o,
                        dptr<T>(H.tmp_res) + o, dptr<T>(L0.t) + o, gate, s, kKcVcycleOther);
    if (L0.ncont < o) {
      const int nz = o - L0.ncont;
      for (int r = 0; r < H.kb; ++r)
        hipLaunchKernelGGL(zero_kernel<T>, dim3(grid_for(nz)), dim3(kThreads), 0, s, nz,
                           dptr<T>(H.tmp_res) + static_cast<int64_t>(r) * L0.n + L0.ncont, gate.all);
    }
    {
      const Range range("V-cycle");
      vcycle(H, 0, dptr<const T>(H.tmp_res), dptr<T>(H.tmp_dz), gate, s);
    }
    hipLaunchKernelGGL(add_kernel<T>, dim3(grid_for(n)), dim3(kThreads), 0, s, static_cast<int>(n),
                       dptr<const T>(H.tmp_dz), z, gate.all);
  }
}

// One application of the block preconditioner, r and z laid out as
// [Omega; Gamma].  On entry Ho.lv[0].t = D^-1 r_O (see start_smoother).
//  * M_L (eq. (8), Algorithm 1): z_O = Q_OO r_O; r_G - A_GO z_O; z_G = Q_GG of it.
//  * M_D (B_D = D^-1 of Section 3.2 made inexact): z_O = Q_OO r_O, z_G = Q_GG r_G.
//  * M_U (B_U = (U D)^-1 made inexact): z_G = Q_GG r_G; r_O - A_OG z_G; z_O = Q_OO of it.
template <typename T>
void apply_ml(Precond<T> &P, const T *r, T *z, Gate gate, hipStream_t s) {
  if (P.n_g == 0 || P.form == MDP_BLOCK_LOWER) {
    apply_q(P.Ho, P.vcycles, r, z, gate, s);  // z_O = Q_OO r_O
    if (P.n_g == 0) return;
    T *rg = dptr<T>(P.rg);
    spmv<kResidScale>(P.Ago, static_cast<const T *>(z), r + P.n_o, dptr<const T>(P.Hg.lv[0].dinv), rg,
                      dptr<T>(P.Hg.lv[0].t), gate, s, kKcVcycleOther);  // r_G - A_GO z_O (and D^-1 of it)
    apply_q(P.Hg, P.vcycles, static_cast<const T *>(rg), z + P.n_o, gate, s);  // z_G = Q_GG r_G
    return;
  }
  if (P.form == MDP_BLOCK_DIAG) {
    apply_q(P.Ho, P.vcycles, r, z, gate, s);  // z_O = Q_OO r_O
    start_smoother(P.Hg, r + P.n_o, gate, s);
    apply_q(P.Hg, P.vcycles, r + P.n_o, z + P.n_o, gate, s);  // z_G = Q_GG r_G
    return;
  }
  start_smoother(P.Hg, r + P.n_o, gate, s);
  apply_q(P.Hg, P.vcycles, r + P.n_o, z + P.n_o, gate, s);  // z_G = Q_GG r_G
  T *ro = dptr<T>(P.rg);
  spmv<kResidScale>(P.Aog, static_cast<const T *>(z + P.n_o), r, dptr<const T>(P.Ho.lv[0].dinv), ro,
                    dptr<T>(P.Ho.lv[0].t), gate, s, kKcVcycleOther);  // r_O - A_OG z_G (and D^-1 of it)
  apply_q(P.Ho, P.vcycles, static_cast<const T *>(ro), z, gate, s);  // z_O = Q_OO of it
}

// Preconditioner for a list of host systems, laid out block-diagonally with
// the level orders plan_o (all systems) and plan_g (systems gsys, which have
// fracture unknowns).  kb > 1: kb right-hand-side blocks of that layout share
// the matrices; the preconditioner's vectors are [Omega blocks; Gamma blocks].
template <typename T>
std::unique_ptr<Precond<T>> upload_precond(const std::vector<const HostSystem *> &sys, const LevelPlan &plan_o,
                                           const LevelPlan &plan_g, const std::vector<int> &gsys,
                                           const mdp_options &opt, bool tails, hipStream_t s, int kb = 1) {
  auto p = std::make_unique<Precond<T>>();
  Keep keep;
  p->vcycles = opt.vcycles;
  p->form = opt.block_form;
  const int form = opt.block_form;
  std::vector<const HHier *> ho, hg;
  for (const HostSystem *h : sys) ho.push_back(&h->Ho);
  for (int q : gsys) hg.push_back(&sys[q]->Hg);
  // batches: row-to-system maps so that stopped pairs' rows are skipped
  std::vector<int> sys_o(sys.size());
  for (size_t q = 0; q < sys.size(); ++q) sys_o[q] = static_cast<int>(q);
  const int nsys = static_cast<int>(sys.size());
  const bool maps = nsys > 1;
  const bool gs = opt.smoother == MDP_SMOOTH_GS;
  upload_hier(ho, plan_o, p->Ho, s, keep, opt.pre_sweeps, opt.post_sweeps, gs, tails, maps ? &sys_o : nullptr, kb,
              nsys);
  p->Ho.is_omega = true;
  const int32_t no1 = p->Ho.n();
  p->n_o = static_cast<int32_t>(p->Ho.nfull());
  if (!gsys.empty()) {
    upload_hier(hg, plan_g, p->Hg, s, keep, opt.pre_sweeps, opt.post_sweeps, gs, tails, maps ? &gsys : nullptr, kb,
                nsys);
    const int32_t ng1 = p->Hg.n();
    p->n_g = static_cast<int32_t>(p->Hg.nfull());
    auto blocks = [&](DCsr<T> &M, int64_t xs, int64_t ys) {
      M.kb = kb;
      M.bxs = xs;
      M.bys = ys;
      M.nsys = nsys;
    };
    std::vector<Piece> pieces;
    for (size_t k = 0; k < gsys.size(); ++k) {
      const int q = gsys[k];
      pieces.emplace_back(&sys[q]->Ago, static_cast<int32_t>(plan_g.off[0][k]),
                          static_cast<int32_t>(plan_o.off[0][q]));
    }
    if (form == MDP_BLOCK_LOWER) {
      upload_csr(concat_blocks(ng1, no1, pieces), p->Ago, s, keep);
      if (maps) p->Ago.rowpair = dptr<const int>(p->Hg.rowpair[0]);
      blocks(p->Ago, no1, ng1);  // x = z_Omega; b, dinv, y = Gamma-sized
      p->rg.alloc(static_cast<size_t>(p->n_g) * sizeof(T));
    } else if (form == MDP_BLOCK_UPPER) {
      std::vector<Piece> up;
      for (size_t k = 0; k < gsys.size(); ++k) {
        const int q = gsys[k];
        up.emplace_back(&sys[q]->Aog, static_cast<int32_t>(plan_o.off[0][q]), static_cast<int32_t>(plan_g.off[0][k]));
      }
      upload_csr(concat_blocks(no1, ng1, up), p->Aog, s, keep);
      if (maps) p->Aog.rowpair = dptr<const int>(p->Ho.rowpair[0]);
      blocks(p->Aog, ng1, no1);  // x = z_Gamma; b, dinv, y = Omega-sized
      p->rg.alloc(static_cast<size_t>(p->n_o) * sizeof(T));
    }
  }
  MDP_HIP(hipStreamSynchronize(s));  // host staging vectors die here
  return p;
}

// ---------------------------------------------------------------------------
// FGMRES over a batch of pairs

// Capture the launches that `enqueue` makes on stream s into an executable
// graph; false (and no graph) if capture or instantiation fails.
template <typename F>
bool capture_step(hipGraphExec_t &out, hipStream_t s, F &&enqueue) {
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  try {
    enqueue();
  } catch (...) {
    (void)hipStreamEndCapture(s, &g);
    if (g) (void)hipGraphDestroy(g);
    throw;
  }
  const bool ok = hipStreamEndCapture(s, &g) == hipSuccess && g != nullptr &&
                  hipGraphInstantiate(&out, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  if (!ok) {
    out = nullptr;
    (void)hipGetLastError();
  }
  return ok;
}

template <typename T>
struct Problem {
  const DCsr<double> *A;
  Precond<T> *P;
  const Layout *L;
  Workspace *ws;
  const mdp_options *opt;
  StepGraphs *graphs;  // where this solve keeps its step graphs (MDP_GRAPHS)
};

// Per-pair norms of v (device) into ws.host_norms (synchronises s).
void pair_norms(Workspace &ws, const Layout &L, const double *v, hipStream_t s) {
  hipLaunchKernelGGL(tile_norm2_kernel, dim3(L.ntiles), dim3(kThreads), 0, s, dptr<const Tile>(L.tiles), v,
                     dptr<double>(ws.npart));
  hipLaunchKernelGGL(pair_norm_kernel, dim3(L.npairs), dim3(kThreads), 0, s, dptr<const double>(ws.npart),
                     dptr<const int>(L.tile_off), dptr<double>(ws.norms));
  MDP_HIP(hipMemcpyAsync(ws.host_norms, ws.norms.get(), sizeof(double) * L.npairs, hipMemcpyDeviceToHost, s));
  MDP_HIP(hipStreamSynchronize(s));
}

// A restart cycle that lowers the true residual by less than this fraction
// makes no progress.  Stagnation is declared after a full cycle (m steps) of
// no progress, or two shorter ones in a row (cycles that the recurrence's
// estimate ended early while the true residual stayed put).
constexpr double kStallFraction = 1e-3;

// Solve A x = b for every pair; bg / xg are in the global layout.  st has one
// entry per pair.  Returns the most severe code (errors before non-convergence).
// retry (optional, one entry per pair) is set to 1 for a pair whose iteration
// produced a NaN/Inf from finite inputs or stagnated: the cases a solve in a
// higher precision may cure.
template <typename T>
int fgmres(Problem<T> &pb, const double *bg, double *xg, bool use_x0, hipStream_t s, mdp_stats *st,
           int *retry = nullptr) {
  Workspace &ws = *pb.ws;
  const Layout &L = *pb.L;
  const DCsr<double> &A = *pb.A;
  Precond<T> &P = *pb.P;
  const mdp_options &opt = *pb.opt;
  const int64_t n = L.n, ld = ws.ld;
  const int m = ws.m, np = L.npairs;
  double *V = dptr<double>(ws.V);
  T *Z = dptr<T>(ws.Z);
  double *w = dptr<double>(ws.w);
  GmresState *dst = dptr<GmresState>(ws.state);
  BatchCtl *ctl = dptr<BatchCtl>(ws.ctl);
  const int *gate_apply = &ctl->skip_all_apply;
  // batches also skip, row by row, the pairs that have stopped
  const Gate g_apply{gate_apply, np > 1 ? static_cast<const GmresState *>(dst) : nullptr};
  const Tile *tiles = dptr<const Tile>(L.tiles);

  std::vector<double> bnorm(np), tol(np), beta(np), est(np, 0.0), scale0(np, 1.0);
  if (np == 1) ws.history.clear();
  std::vector<int> iters(np, 0), cycles(np, 0), code(np, MDP_OK), active(np, 0), kmax_h(np, 0), stall(np, 0);
  if (retry) std::fill(retry, retry + np, 0);
  pair_norms(ws, L, bg, s);
  for (int p = 0; p < np; ++p) {
    bnorm[p] = ws.host_norms[p];
    tol[p] = opt.rtol * bnorm[p];
    if (!std::isfinite(bnorm[p])) code[p] = MDP_ENAN;
  }
  if (!use_x0) MDP_HIP(hipMemsetAsync(xg, 0, n * sizeof(double), s));
  if (use_x0) {
    spmv<kResid>(A, static_cast<const double *>(xg), bg, cnull<double>(), V, mnull<double>(), Gate{}, s);
    pair_norms(ws, L, V, s);
    for (int p = 0; p < np; ++p) beta[p] = ws.host_norms[p];
  } else {
    MDP_HIP(hipMemcpyAsync(V, bg, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    beta = bnorm;
  }

  // With MDP_GRAPHS, each step is replayed from a graph captured on its first
  // use (not on the legacy stream, which cannot be captured, and not while
  // timers run).  Graphs captured with another workspace are dropped.
  StepGraphs *sg = pb.graphs;
  bool use_graphs = sg && (opt.flags & MDP_GRAPHS) && !ktimer_any_on() && !sg->failed && s != nullptr;
  if (use_graphs && (sg->ws != &ws || sg->ws_gen != ws.gen || sg->exec.size() != static_cast<size_t>(2 * (m + 1)))) {
    sg->clear();
    sg->exec.assign(2 * (m + 1), nullptr);
    sg->ws = &ws;
    sg->ws_gen = ws.gen;
  }
  while (true) {
    int nactive = 0, kmax_all = 0;
    for (int p = 0; p < np; ++p) {
      if (code[p] == MDP_OK && !std::isfinite(beta[p])) code[p] = MDP_ENAN;
      active[p] = code[p] == MDP_OK && bnorm[p] > 0.0 && beta[p] > tol[p] && iters[p] < opt.max_iter;
      kmax_h[p] = std::min(m, opt.max_iter - iters[p]);
      if (active[p]) {
        ++nactive;
        kmax_all = std::max(kmax_all, kmax_h[p]);
      }
    }
    if (nactive == 0) break;
    const Range cycle_range("fgmres cycle");
    MDP_HIP(hipMemcpyAsync(ws.active.get(), active.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
    MDP_HIP(hipMemcpyAsync(ws.kmaxp.get(), kmax_h.data(), sizeof(int) * np, hipMemcpyHostToDevice, s));
    MDP_HIP(hipMemcpyAsync(ws.tolp.get(), tol.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    if constexpr (!std::is_same<T, double>::value) {
      // mixed: the cycle's first FP32 preconditioner input is the residual / beta
      for (int p = 0; p < np; ++p) scale0[p] = active[p] && beta[p] > 0.0 ? 1.0 / beta[p] : 1.0;
      MDP_HIP(hipMemcpyAsync(ws.scale0.get(), scale0.data(), sizeof(double) * np, hipMemcpyHostToDevice, s));
    }
    hipLaunchKernelGGL(cycle_init_kernel, dim3(np), dim3(64), 0, s, dst, ctl, np, nactive,
                       dptr<const int>(ws.active), dptr<double>(ws.g), ws.ldv);
    // V[:, 0] holds every pair's residual at the cycle start, unnormalised.
    // Steps 0..kmax-1 apply the preconditioner; step kmax (if reached) only
    // finalises the last Hessenberg column.
    int counted = 0;  // steps whose algorithmic bytes were counted
    // One Arnoldi step: preconditioner input, M z_j, w = A z_j, the fused
    // reduction, the per-pair scalars and the update pass, then the control
    // word to the host.  Every argument is fixed by (j, zcol) for a given
    // workspace, so single-system solves capture the step once and replay it.
    auto enqueue_step = [&](int j, int zcol) {
      T *zj = Z + zcol * ld;
      const double *uj = V + j * ld;
      const T *pin;
      // The preconditioner input of step j > 0 was written by the update pass
      // of step j - 1 (see NextInput); the first step of a cycle prepares it here.
      if constexpr (std::is_same<T, double>::value) {
        pin = uj;
        if (j == 0) start_smoother(P.Ho, pin, g_apply, s);
      } else {
        pin = dptr<T>(ws.rin);
        if (j == 0) {
          T *rin = dptr<T>(ws.rin);
          const int no = P.n_o;
          const bool need_t = !P.Ho.dense_only();
          timed_launch(kKcOther, s, 12.0 * n + 8.0 * no, [&] {
            hipLaunchKernelGGL(cast_start_kernel, dim3(L.ntiles), dim3(kThreads), 0, s, tiles,
                               static_cast<int64_t>(no), uj, dptr<const double>(ws.scale0), rin,
                               dptr<const float>(P.Ho.lv[0].dinv), need_t ? dptr<float>(P.Ho.lv[0].t) : nullptr,
                               gate_apply);
          });
        }
      }
      {
        const Range r("M_L apply");
        apply_ml(P, pin, zj, g_apply, s);
      }
      const Range r("Arnoldi step");
      spmv<kPlain>(A, static_cast<const T *>(zj), cnull<double>(), cnull<double>(), w, mnull<double>(), g_apply,
                   s, kKcOuterSpmv);
      const int nv = 2 * j + 3;
      timed_launch(kKcArnoldiDot, s, 8.0 * n * (j + 2), [&] {
        hipLaunchKernelGGL(dcgs_reduce_kernel, dim3(L.ntiles), dim3(kThreads), 0, s, tiles, L.ntiles, j,
                           static_cast<const double *>(V), ld, static_cast<const double *>(w),
                           dptr<double>(ws.partial), static_cast<const GmresState *>(dst));
      });
      timed_launch(kKcOther, s, 8.0 * nv * L.ntiles, [&] {
        hipLaunchKernelGGL(pair_sums_kernel, dim3(nv, np), dim3(kThreads), 0, s, nv, dptr<const double>(ws.partial),
                           L.ntiles, dptr<const int>(L.tile_off), dptr<double>(ws.sums), ws.sstride,
                           static_cast<const GmresState *>(dst));
      });
      timed_launch(kKcOther, s, 0.0, [&] {
        hipLaunchKernelGGL(dcgs_finalize_kernel, dim3(np), dim3(64), 0, s, dst, ctl, np, j,
                           dptr<const int>(ws.kmaxp), dptr<const double>(ws.tolp), dptr<const double>(ws.sums),
                           ws.sstride, dptr<double>(ws.hprev), dptr<DcgsCoef>(ws.coef), dptr<double>(ws.Hr), m + 1,
                           m, dptr<double>(ws.cs), dptr<double>(ws.sn), dptr<double>(ws.g), dptr<double>(ws.hist),
                           ws.ldv);
      });
      // the update pass also writes step j + 1's preconditioner input and
      // sends this step's control word to the host
      NextInput nin{};
      double next_bytes = 0.0;
      const bool need_t = !P.Ho.dense_only();
      if constexpr (std::is_same<T, double>::value) {
        if (need_t) {
          nin.t64 = dptr<double>(P.Ho.lv[0].t);
          nin.dinv64 = dptr<const double>(P.Ho.lv[0].dinv);
          next_bytes = 16.0 * P.n_o;
        }
      } else {
        nin.rin = dptr<float>(ws.rin);
        next_bytes = 4.0 * n;
        if (need_t) {
          nin.t32 = dptr<float>(P.Ho.lv[0].t);
          nin.dinv32 = dptr<const float>(P.Ho.lv[0].dinv);
          next_bytes += 8.0 * P.n_o;
        }
      }
      nin.n_o = P.n_o;
      nin.host_ctl = ws.host_ctl_dev + j;
      nin.ctl = ctl;
      timed_launch(kKcArnoldiAxpy, s, 8.0 * n * (j + 4) + next_bytes, [&] {
        hipLaunchKernelGGL(dcgs_update_kernel, dim3(L.ntiles), dim3(kThreads), 0, s, tiles, j, V, ld,
                           static_cast<const double *>(w), dptr<const DcgsCoef>(ws.coef),
                           static_cast<const GmresState *>(dst), nin);
      });
    };
    for (int j = 0; j <= kmax_all; ++j) {
      const KtBytes kt_before = ktimer_bytes();
      ++counted;
      const int zcol = std::min(j, kmax_all - 1);
      if (use_graphs) {
        hipGraphExec_t &ge = sg->exec[(zcol == j ? 0 : m + 1) + j];
        if (!ge && !capture_step(ge, s, [&] { enqueue_step(j, zcol); })) {
          sg->failed = true;
          use_graphs = false;
        }
        if (ge) MDP_HIP(hipGraphLaunch(ge, s));
      }
      if (!use_graphs) enqueue_step(j, zcol);
      MDP_HIP(hipEventRecord(ws.ev[j], s));
      if (j >= 1) {
        MDP_HIP(hipEventSynchronize(ws.ev[j - 1]));
        if (ws.host_ctl[j - 1].all_done) {
          ktimer_restore_bytes(kt_before);  // step j was queued after the cycle ended: a no-op
          --counted;
          break;
        }
      }
    }
    MDP_HIP(hipGetLastError());
    MDP_HIP(hipMemcpyAsync(ws.host_state, dst, sizeof(GmresState) * np, hipMemcpyDeviceToHost, s));
    if (np == 1)  // this cycle's residual estimates, read after the synchronisation below
      MDP_HIP(hipMemcpyAsync(ws.host_hist, ws.hist.get(), sizeof(double) * m, hipMemcpyDeviceToHost, s));
    hipLaunchKernelGGL(backsolve_kernel, dim3(np), dim3(64), 0, s, static_cast<const GmresState *>(dst),
                       dptr<const double>(ws.Hr), m + 1, m, dptr<const double>(ws.g), dptr<double>(ws.y), ws.ldv);
    timed_launch(kKcOther, s, 16.0 * n, [&] {
      hipLaunchKernelGGL((update_x_kernel<T>), dim3(L.ntiles), dim3(kThreads), 0, s, tiles,
                         static_cast<const T *>(Z), ld, dptr<const double>(ws.y), ws.ldv,
                         static_cast<const GmresState *>(dst), dptr<const int>(ws.active), xg);
    });
    spmv<kResid>(A, static_cast<const double *>(xg), bg, cnull<double>(), V, mnull<double>(), Gate{}, s);
    pair_norms(ws, L, V, s);  // synchronises: host_state is valid too
    if (np > 1 && (ktimer_on(kKcArnoldiDot) || ktimer_on(kKcArnoldiAxpy))) {
      // The Arnoldi passes were counted as if every pair ran every step;
      // pairs that had finished skip their tiles.  Pair p (k steps in this
      // cycle) reduces at steps 0..k and updates at steps 0..k-1.
      double over_dot = 0.0, over_axpy = 0.0;
      for (int j = 0; j < counted; ++j) {
        int64_t red = 0, upd = 0;
        for (int p = 0; p < np; ++p) {
          if (!active[p]) continue;
          const int k = ws.host_state[p].k;
          if (k >= j) red += L.rows[p];
          if (k > j) upd += L.rows[p];
        }
        over_dot += 8.0 * (j + 2) * static_cast<double>(n - red);
        over_axpy += 8.0 * (j + 4) * static_cast<double>(n - upd);
      }
      ktimer_add_bytes(kKcArnoldiDot, -over_dot);
      ktimer_add_bytes(kKcArnoldiAxpy, -over_axpy);
    }
    for (int p = 0; p < np; ++p) {
      if (!active[p]) continue;
      const GmresState &gs = ws.host_state[p];
      if (gs.nan) {
        code[p] = MDP_ENAN;
        if (retry) retry[p] = 1;
      }
      iters[p] += gs.k;
      est[p] = gs.est;
      ++cycles[p];
      if (np == 1 && bnorm[p] > 0.0)
        for (int i = 0; i < gs.k && i < m; ++i) ws.history.push_back(ws.host_hist[i] / bnorm[p]);
      const double b_new = ws.host_norms[p];
      if (code[p] == MDP_OK && b_new > tol[p] && iters[p] < opt.max_iter) {
        if (b_new > (1.0 - kStallFraction) * beta[p])
          stall[p] += gs.k >= m ? 2 : 1;
        else
          stall[p] = 0;
        if (stall[p] >= 2) {
          code[p] = MDP_STAGNATED;
          if (retry) retry[p] = 1;
        }
      }
      beta[p] = b_new;
    }
  }
  MDP_HIP(hipGetLastError());
  int worst = MDP_OK;
  for (int p = 0; p < np; ++p) {
    mdp_stats o{};
    o.iters = iters[p];
    o.restarts = std::max(cycles[p] - 1, 0);
    if (bnorm[p] == 0.0) {
      o.converged = code[p] == MDP_OK;
    } else {
      o.rel_res_true = beta[p] / bnorm[p];
      o.rel_res_est = (cycles[p] > 0 ? est[p] : beta[p]) / bnorm[p];
      o.converged = (code[p] == MDP_OK && beta[p] <= tol[p]) ? 1 : 0;
    }
    if (code[p] == MDP_OK && !o.converged) code[p] = MDP_NOT_CONVERGED;
    o.status = code[p];
    if (st) st[p] = o;
    if (code[p] < 0) {
      if (worst >= 0 || code[p] < worst) worst = code[p];
    } else if (worst >= 0 && code[p] > worst) {
      worst = code[p];
    }
  }
  return worst;
}

}  // namespace

// ---------------------------------------------------------------------------

void Layout::build(const std::vector<std::vector<std::pair<int64_t, int64_t>>> &ranges, int64_t n_total,
                   hipStream_t s) {
  npairs = static_cast<int>(ranges.size());
  n = n_total;
  rows.assign(static_cast<size_t>(npairs), 0);
  for (int p = 0; p < npairs; ++p)
    for (const auto &r : ranges[p]) rows[p] += r.second;
  std::vector<int32_t> off;
  const std::vector<Tile> tl = plan_tiles(ranges, off);
  ntiles = static_cast<int>(tl.size());
  upload_vec(tiles, tl, s);
  upload_vec(tile_off, off, s);
  MDP_HIP(hipStreamSynchronize(s));
}

size_t Workspace::bytes_for(int64_t n, int m_, int np, int nt, size_t tsz_, bool perm) {
  const size_t ld_ = static_cast<size_t>(padded_ld(n));
  const size_t ldv_ = static_cast<size_t>(m_) + 2, ss = 2 * (static_cast<size_t>(m_) + 1) + 4;
  const size_t npz = static_cast<size_t>(np), ntz = static_cast<size_t>(std::max(nt, 1));
  size_t b = ld_ * 8 * (m_ + 1) + ld_ * tsz_ * m_ + ld_ * 8 + ld_ * tsz_;  // V, Z, w, rin
  if (perm) b += 2 * ld_ * 8;                                             // bp, xp
  b += 6 * npz * ldv_ * 8 + npz * (m_ + 1) * m_ * 8 + npz * sizeof(DcgsCoef) + npz * ss * 8;
  b += (2 * (m_ + 1) + 3) * ntz * 8 + ntz * 8 + npz * sizeof(GmresState) + sizeof(BatchCtl);
  b += npz * (4 + 8 + 8 + 4 + 8);  // kmaxp, tolp, scale0, active, norms
  return b;
}

bool Workspace::fits(int64_t n, int m_, int np, int nt, size_t tsz_) const {
  return allocated() && ld >= n && m == m_ && npairs >= np && ntiles >= nt && tsz >= tsz_ && bp.get() && xp.get();
}

void Workspace::alloc(int64_t n, int m_, int np, int nt, size_t tsz_, hipStream_t s) {
  static std::atomic<uint64_t> generations{0};
  gen = ++generations;
  m = m_;
  tsz = tsz_;
  npairs = np;
  ntiles = std::max(nt, 1);
  ld = padded_ld(n);
  ldv = m + 2;
  sstride = 2 * (m + 1) + 4;
  const size_t col8 = static_cast<size_t>(ld) * sizeof(double);
  V.alloc(col8 * (m + 1));
  Z.alloc(static_cast<size_t>(ld) * tsz * m);
  w.alloc(col8);
  rin.alloc(static_cast<size_t>(ld) * tsz);
  // whole-batch kernels also read the columns of pairs that stopped early:
  // start from finite values
  MDP_HIP(hipMemsetAsync(V.get(), 0, V.bytes(), s));
  MDP_HIP(hipMemsetAsync(Z.get(), 0, Z.bytes(), s));
  const size_t pv = static_cast<size_t>(np) * ldv * sizeof(double);
  for (DevMem *d : {&cs, &sn, &g, &y, &hist, &hprev}) d->alloc(pv);
  Hr.alloc(static_cast<size_t>(np) * (m + 1) * m * sizeof(double));
  coef.alloc(static_cast<size_t>(np) * sizeof(DcgsCoef));
  sums.alloc(static_cast<size_t>(np) * sstride * sizeof(double));
  partial.alloc(static_cast<size_t>(2 * (m + 1) + 3) * ntiles * sizeof(double));
  npart.alloc(static_cast<size_t>(ntiles) * sizeof(double));
  state.alloc(static_cast<size_t>(np) * sizeof(GmresState));
  ctl.alloc(sizeof(BatchCtl));
  kmaxp.alloc(static_cast<size_t>(np) * sizeof(int));
  tolp.alloc(static_cast<size_t>(np) * sizeof(double));
  scale0.alloc(static_cast<size_t>(np) * sizeof(double));
  active.alloc(static_cast<size_t>(np) * sizeof(int));
  norms.alloc(static_cast<size_t>(np) * sizeof(double));
  // written by the update kernel through its device address (mapped, coherent)
  MDP_HIP(hipHostMalloc(reinterpret_cast<void **>(&host_ctl), (m + 2) * sizeof(BatchCtl),
                        hipHostMallocMapped | hipHostMallocCoherent));
  MDP_HIP(hipHostGetDevicePointer(reinterpret_cast<void **>(&host_ctl_dev), host_ctl, 0));
  MDP_HIP(hipHostMalloc(reinterpret_cast<void **>(&host_state), np * sizeof(GmresState), hipHostMallocDefault));
  MDP_HIP(hipHostMalloc(reinterpret_cast<void **>(&host_norms), np * sizeof(double), hipHostMallocDefault));
  MDP_HIP(hipHostMalloc(reinterpret_cast<void **>(&host_hist), (m + 2) * sizeof(double), hipHostMallocDefault));
  ev.resize(static_cast<size_t>(m) + 2);
  for (auto &e : ev) MDP_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  MDP_HIP(hipStreamSynchronize(s));
}

void StepGraphs::clear() {
  for (hipGraphExec_t g : exec)
    if (g) (void)hipGraphExecDestroy(g);
  exec.clear();
  ws = nullptr;
  failed = false;
}

hipStream_t Workspace::own_stream() {
  if (!own) {
    MDP_HIP(hipStreamCreateWithFlags(&own, hipStreamNonBlocking));
    MDP_HIP(hipEventCreateWithFlags(&handoff, hipEventDisableTiming));
  }
  return own;
}

void Workspace::release() {
  graphs.clear();
  graphs64.clear();
  tsz = 0;
  if (handoff) (void)hipEventDestroy(handoff);
  if (own) (void)hipStreamDestroy(own);
  handoff = nullptr;
  own = nullptr;
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  ev.clear();
  if (host_ctl) (void)hipHostFree(host_ctl);
  if (host_state) (void)hipHostFree(host_state);
  if (host_norms) (void)hipHostFree(host_norms);
  if (host_hist) (void)hipHostFree(host_hist);
  host_hist = nullptr;
  host_ctl = nullptr;
  host_ctl_dev = nullptr;
  host_state = nullptr;
  host_norms = nullptr;
  for (DevMem *d : {&V, &Z, &w, &rin, &bp, &xp, &Hr, &cs, &sn, &g, &y, &hist, &hprev, &coef, &sums, &partial, &npart,
                    &state, &ctl, &kmaxp, &tolp, &scale0, &active, &norms})
    d->reset();
}

size_t Workspace::device_bytes() const {
  size_t b = 0;
  for (const DevMem *d : {&V, &Z, &w, &rin, &bp, &xp, &Hr, &cs, &sn, &g, &y, &hist, &hprev, &coef, &sums, &partial,
                          &npart, &state, &ctl, &kmaxp, &tolp, &scale0, &active, &norms})
    b += d->bytes();
  return b;
}

size_t Solver::workspace_bytes_needed() const {
  const size_t ld = static_cast<size_t>(padded_ld(n));
  const size_t tsz = opt.precision == MDP_MIXED ? sizeof(float) : sizeof(double);
  const size_t m = static_cast<size_t>(opt.restart);
  size_t b = ld * 8 * (m + 1) + ld * tsz * m + ld * 8 + ld * tsz;  // V, Z, w, rin
  if (!host.identity) b += 2 * ld * 8;
  return b + (size_t{1} << 20);  // small per-pair arrays
}

void Solver::ensure_workspace(hipStream_t s) {
  if (ws.allocated()) return;
  const size_t tsz = opt.precision == MDP_MIXED ? sizeof(float) : sizeof(double);
  ws.alloc(n, opt.restart, 1, layout.ntiles, tsz, s);
  if (!host.identity) {
    ws.bp.alloc(static_cast<size_t>(ws.ld) * sizeof(double));
    ws.xp.alloc(static_cast<size_t>(ws.ld) * sizeof(double));
  }
}

void Solver::upload(hipStream_t s) {
  const AutotuneScope tune((opt.flags & MDP_NO_AUTOTUNE) == 0);
  const auto t0 = std::chrono::steady_clock::now();
  n = host.n;
  n_o = host.n_o;
  n_g = host.n_g;
  Keep keep;
  upload_csr(host.A, A, s, keep);
  if (!host.identity) upload_vec(perm, host.perm, s);
  const std::vector<const HostSystem *> sys{&host};
  // each hierarchy's dense tail for this handle's smoothing (none with
  // Gauss-Seidel, whose sweeps the tail does not model)
  for (HHier *hh : {&host.Ho, &host.Hg}) {
    if (opt.smoother == MDP_SMOOTH_GS)
      clear_tail(*hh);
    else
      form_tail(*hh, opt.pre_sweeps, opt.post_sweeps, opt.max_dense);
  }
  const LevelPlan po = plan_levels({&host.Ho}, true);
  const LevelPlan pg = n_g > 0 ? plan_levels({&host.Hg}, true) : LevelPlan{};
  const std::vector<int> gp = n_g > 0 ? std::vector<int>{0} : std::vector<int>{};
  if (opt.precision == MDP_MIXED)
    pc32 = upload_precond<float>(sys, po, pg, gp, opt, true, s);
  else
    pc64 = upload_precond<double>(sys, po, pg, gp, opt, true, s);
  layout.build({{{0, n}}}, n, s);
  const size_t tsz = opt.precision == MDP_MIXED ? sizeof(float) : sizeof(double);
  ws.alloc(n, opt.restart, 1, layout.ntiles, tsz, s);
  if (!host.identity) {
    ws.bp.alloc(static_cast<size_t>(ws.ld) * sizeof(double));
    ws.xp.alloc(static_cast<size_t>(ws.ld) * sizeof(double));
  }
  MDP_HIP(hipStreamSynchronize(s));
  on_device = true;
  if (std::getenv("MDP_SETUP_VERBOSE"))
    std::fprintf(stderr, "[mdp] device upload %.3f s\n",
                 std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
}

int Solver::solve(const double *b, double *x, hipStream_t s, mdp_stats *st, bool fp64_only) {
  const Range range("mdp_solve");
  const auto t0 = std::chrono::steady_clock::now();
  ensure_workspace(s);
  // The legacy stream cannot be captured: a solve handed it runs on the
  // workspace's own stream, after the caller's earlier work on s.
  const hipStream_t caller = s;
  if (s == nullptr && (opt.flags & MDP_GRAPHS) && !ktimer_any_on() && !ws.graphs.failed) {
    s = ws.own_stream();
    MDP_HIP(hipEventRecord(ws.handoff, caller));
    MDP_HIP(hipStreamWaitEvent(s, ws.handoff, 0));
  }
  const bool use_x0 = (opt.flags & MDP_USE_X0) != 0;
  const double *bp = b;
  double *xp = x;
  if (!host.identity) {
    const int g = grid_for(n);
    hipLaunchKernelGGL(permute_kernel<true>, dim3(g), dim3(kThreads), 0, s, n, dptr<const int>(perm), b,
                       dptr<double>(ws.bp));
    bp = dptr<const double>(ws.bp);
    xp = dptr<double>(ws.xp);
    if (use_x0)
      hipLaunchKernelGGL(permute_kernel<true>, dim3(g), dim3(kThreads), 0, s, n, dptr<const int>(perm), x, xp);
  }
  mdp_stats out{};
  int rc;
  if (opt.precision == MDP_MIXED && fp64_only) {
    // a column whose mixed solve failed elsewhere (a four-column group)
    ensure_fp64(s);
    Problem<double> p64{&A, pc64.get(), &layout, &ws, &opt, &ws.graphs64};
    rc = fgmres<double>(p64, bp, xp, false, s, &out);
    out.fallback = 1;
  } else if (opt.precision == MDP_MIXED) {
    Problem<float> pb{&A, pc32.get(), &layout, &ws, &opt, &ws.graphs};
    int retry = 0;
    rc = fgmres<float>(pb, bp, xp, use_x0, s, &out, &retry);
    if (retry && (opt.flags & MDP_FALLBACK_FP64)) {
      // the FP32 preconditioner failed this column: solve it again from zero
      // with the FP64 one (the graphs of the FP32 steps do not apply to it)
      const int32_t it_mixed = out.iters, cyc_mixed = out.restarts + 1;
      ensure_fp64(s);
      Problem<double> p64{&A, pc64.get(), &layout, &ws, &opt, &ws.graphs64};
      rc = fgmres<double>(p64, bp, xp, false, s, &out);
      out.iters += it_mixed;
      out.restarts += cyc_mixed;
      out.fallback = 1;
    }
  } else {
    Problem<double> pb{&A, pc64.get(), &layout, &ws, &opt, &ws.graphs};
    rc = fgmres<double>(pb, bp, xp, use_x0, s, &out);
  }
  if (!host.identity)
    hipLaunchKernelGGL(permute_kernel<false>, dim3(grid_for(n)), dim3(kThreads), 0, s, n, dptr<const int>(perm),
                       static_cast<const double *>(xp), x);
  MDP_HIP(hipGetLastError());
  MDP_HIP(hipStreamSynchronize(s));
  out.solve_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  out.setup_ms = setup_ms;
  if (st) *st = out;
  return rc;
}

void Solver::ensure_fp64(hipStream_t s) {
  if (!pc64) {
    const AutotuneScope tune((opt.flags & MDP_NO_AUTOTUNE) == 0);
    const std::vector<const HostSystem *> sys{&host};
    const LevelPlan po = plan_levels({&host.Ho}, true);
    const LevelPlan pg = n_g > 0 ? plan_levels({&host.Hg}, true) : LevelPlan{};
    const std::vector<int> gp = n_g > 0 ? std::vector<int>{0} : std::vector<int>{};
    pc64 = upload_precond<double>(sys, po, pg, gp, opt, true, s);
  }
  if (ws.tsz < sizeof(double)) {
    // Z holds FP64 directions from now on (FP32 solves use the wider array as
    // it is).  Only Z moves: the solve's permuted b and x, its stream and its
    // events stay; graphs captured with the old Z are dropped.
    MDP_HIP(hipStreamSynchronize(s));
    ws.graphs.clear();
    ws.graphs64.clear();
    ws.Z.alloc(static_cast<size_t>(ws.ld) * sizeof(double) * ws.m);
    MDP_HIP(hipMemsetAsync(ws.Z.get(), 0, ws.Z.bytes(), s));
    ws.tsz = sizeof(double);
    ++ws.gen;
  }
}

void Solver::apply(int op, const double *x, double *y, hipStream_t s) {
  const Range range("mdp_apply");
  ensure_workspace(s);
  enqueue_apply(op, x, y, s, dptr<float>(ws.rin), dptr<float>(ws.Z));
  MDP_HIP(hipStreamSynchronize(s));
}

void Solver::enqueue_apply(int op, const double *x, double *y, hipStream_t s, float *in, float *out) {
  const int64_t nn = n;
  switch (op) {
    case MDP_OP_A:
      spmv<kPlain>(A, x, cnull<double>(), cnull<double>(), y, mnull<double>(), Gate{}, s);
      break;
    case MDP_OP_ML:
    case MDP_OP_QOO:
    case MDP_OP_QGG: {
      const int64_t len = op == MDP_OP_ML ? nn : (op == MDP_OP_QOO ? n_o : n_g);
      if (len == 0) break;
      if (opt.precision == MDP_MIXED) {
        hipLaunchKernelGGL((scale_copy_kernel<double, float>), dim3(grid_for(len)), dim3(kThreads), 0, s, len, x,
                           cnull<double>(), in, nullptr);
        auto &H = op == MDP_OP_QGG ? pc32->Hg : pc32->Ho;
        start_smoother(H, static_cast<const float *>(in), Gate{}, s);
        if (op == MDP_OP_ML)
          apply_ml(*pc32, static_cast<const float *>(in), out, Gate{}, s);
        else
          apply_q(H, pc32->vcycles, static_cast<const float *>(in), out, Gate{}, s);
        hipLaunchKernelGGL((scale_copy_kernel<float, double>), dim3(grid_for(len)), dim3(kThreads), 0, s, len,
                           static_cast<const float *>(out), cnull<double>(), y, nullptr);
      } else {
        auto &H = op == MDP_OP_QGG ? pc64->Hg : pc64->Ho;
        start_smoother(H, x, Gate{}, s);
        if (op == MDP_OP_ML)
          apply_ml(*pc64, x, y, Gate{}, s);
        else
          apply_q(H, pc64->vcycles, x, y, Gate{}, s);
      }
      break;
    }
    default:
      raise(MDP_EINVAL, "unknown operator");
  }
  MDP_HIP(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Batches

// Vector blocks of a batch: kMultiRhs when every system in it has exactly
// kMultiRhs right-hand sides, else 1 (every pair its own block).
int batch_blocks(const std::vector<const Solver *> &pairs) {
  std::map<const Solver *, int> count;
  for (const Solver *p : pairs) ++count[p];
  for (const auto &c : count)
    if (c.second != kMultiRhs) return 1;
  return kMultiRhs;
}

void Batch::build(const std::vector<const Solver *> &pairs, hipStream_t s, bool alloc_ws) {
  const AutotuneScope tune(!pairs.empty() && (pairs[0]->opt.flags & MDP_NO_AUTOTUNE) == 0);
  sys = pairs;
  npairs = static_cast<int>(pairs.size());
  opt = pairs[0]->opt;
  // The block's systems, and the internal pair order: pair r * nsys + k is
  // the r-th right-hand side of system k (with kb = 1, every pair is a system).
  kb = batch_blocks(pairs);
  std::vector<const Solver *> bsys;
  order.assign(static_cast<size_t>(npairs), -1);
  if (kb == 1) {
    bsys = pairs;
    for (int q = 0; q < npairs; ++q) order[q] = q;
  } else {
    std::map<const Solver *, int> index;
    std::vector<int> sys_of(static_cast<size_t>(npairs));
    for (int p = 0; p < npairs; ++p) {
      auto it = index.find(pairs[p]);
      if (it == index.end()) {
        it = index.emplace(pairs[p], static_cast<int>(bsys.size())).first;
        bsys.push_back(pairs[p]);
      }
      sys_of[p] = it->second;
    }
    std::vector<int> seen(bsys.size(), 0);
    const int ns = static_cast<int>(bsys.size());
    for (int p = 0; p < npairs; ++p) order[seen[sys_of[p]]++ * ns + sys_of[p]] = p;
  }
  nsys = static_cast<int>(bsys.size());
  std::vector<const HostSystem *> hsys;
  std::vector<const HHier *> ho, hg;
  std::vector<int> gsys;
  for (int k = 0; k < nsys; ++k) {
    hsys.push_back(&bsys[k]->host);
    ho.push_back(&bsys[k]->host.Ho);
    if (bsys[k]->host.n_g > 0) {
      gsys.push_back(k);
      hg.push_back(&bsys[k]->host.Hg);
    }
  }
  // dense tails only for plans of one system (a four-column group): over many
  // different systems the tails' dense matrices outweigh the shared launches
  // they save
  const bool tails = bsys.size() == 1;
  const LevelPlan po = plan_levels(ho, tails);
  const LevelPlan pg = gsys.empty() ? LevelPlan{} : plan_levels(hg, tails);
  const int64_t no1 = po.n[0], ng1 = gsys.empty() ? 0 : pg.n[0];
  if (kb * (no1 + ng1) > std::numeric_limits<int32_t>::max()) raise(MDP_EINVAL, "batch exceeds int32 indexing");
  n_o = static_cast<int32_t>(kb * no1);
  n_g = static_cast<int32_t>(kb * ng1);
  n = n_o + n_g;
  // global row of (internal pair q, internal index): Omega rows of block
  // q / nsys in the S~ hierarchies' level-0 order, then Gamma rows of that
  // block in the A_GG hierarchies' level-0 order
  std::vector<int64_t> goff_g(static_cast<size_t>(nsys), -1);
  for (size_t k = 0; k < gsys.size(); ++k) goff_g[gsys[k]] = pg.off[0][k];
  auto omega_at = [&](int q) { return (q / nsys) * no1 + po.off[0][q % nsys]; };
  auto gamma_at = [&](int q) { return n_o + (q / nsys) * ng1 + goff_g[q % nsys]; };
  std::vector<int32_t> gidx_h(static_cast<size_t>(n)), gpair_h(static_cast<size_t>(n));
  std::vector<std::vector<std::pair<int64_t, int64_t>>> ranges(static_cast<size_t>(npairs));
  HCsr Ag = HCsr::empty(n, n);
  {
    std::vector<int32_t> rowlen(static_cast<size_t>(n), 0);
    for (int q = 0; q < npairs; ++q) {
      const HostSystem &h = *hsys[q % nsys];
      const int64_t oo = omega_at(q), og = gamma_at(q);
      ranges[q].push_back({oo, h.n_o});
      if (h.n_g > 0) ranges[q].push_back({og, h.n_g});
      for (int32_t i = 0; i < h.n; ++i) {
        const int64_t g = i < h.n_o ? oo + i : og + (i - h.n_o);
        rowlen[g] = h.A.ptr[i + 1] - h.A.ptr[i];
        gidx_h[g] = h.perm[i];
        gpair_h[g] = q;
      }
    }
    for (int32_t i = 0; i < n; ++i) Ag.ptr[i + 1] = Ag.ptr[i] + rowlen[i];
    Ag.col.resize(static_cast<size_t>(Ag.ptr[n]));
    Ag.val.resize(static_cast<size_t>(Ag.ptr[n]));
    for (int q = 0; q < npairs; ++q) {
      const HostSystem &h = *hsys[q % nsys];
      const int64_t oo = omega_at(q), og = gamma_at(q);
      auto gmap = [&](int32_t i) { return static_cast<int32_t>(i < h.n_o ? oo + i : og + (i - h.n_o)); };
      for (int32_t i = 0; i < h.n; ++i) {
        int32_t k2 = Ag.ptr[gmap(i)];
        for (int32_t k = h.A.ptr[i]; k < h.A.ptr[i + 1]; ++k, ++k2) {
          Ag.col[k2] = gmap(h.A.col[k]);
          Ag.val[k2] = h.A.val[k];
        }
      }
    }
  }
  Keep keep;
  upload_csr(Ag, A, s, keep);
  upload_vec(gidx, keep.put(std::move(gidx_h)), s);
  upload_vec(gpair, keep.put(std::move(gpair_h)), s);
  if (npairs > 1) A.rowpair = dptr<const int>(gpair);
  if (opt.precision == MDP_MIXED)
    pc32 = upload_precond<float>(hsys, po, pg, gsys, opt, tails, s, kb);
  else
    pc64 = upload_precond<double>(hsys, po, pg, gsys, opt, tails, s, kb);
  layout.build(ranges, n, s);
  if (std::getenv("MDP_SETUP_VERBOSE"))
    std::fprintf(stderr, "[mdp] batch: %d pairs, %d right-hand-side blocks of %d systems, n=%d\n", npairs, kb, nsys,
                 n);
  if (alloc_ws) {
    const size_t tsz = opt.precision == MDP_MIXED ? sizeof(float) : sizeof(double);
    ws.alloc(n, opt.restart, npairs, layout.ntiles, tsz, s);
    ws.bp.alloc(static_cast<size_t>(ws.ld) * sizeof(double));
    ws.xp.alloc(static_cast<size_t>(ws.ld) * sizeof(double));
  }
  MDP_HIP(hipStreamSynchronize(s));
}

int Batch::solve(const std::vector<PairIO> &io, hipStream_t s, mdp_stats *st) {
  const Range range("mdp_solve_batch");
  const auto t0 = std::chrono::steady_clock::now();
  const bool use_x0 = (opt.flags & MDP_USE_X0) != 0;
  Workspace &W = wsp ? *wsp : ws;
  if (!W.fits(n, opt.restart, npairs, layout.ntiles, opt.precision == MDP_MIXED ? sizeof(float) : sizeof(double)))
    raise(MDP_EINVAL, "batch workspace missing or too small");
  // As for single solves: graph replay cannot capture the legacy stream, so
  // the batch then runs on the workspace's own stream after the caller's work.
  const hipStream_t caller = s;
  if (s == nullptr && (opt.flags & MDP_GRAPHS) && !ktimer_any_on() && !graphs.failed) {
    s = W.own_stream();
    MDP_HIP(hipEventRecord(W.handoff, caller));
    MDP_HIP(hipStreamWaitEvent(s, W.handoff, 0));
  }
  std::vector<const double *> bptr(static_cast<size_t>(npairs));
  std::vector<double *> xptr(static_cast<size_t>(npairs));
  for (int q = 0; q < npairs; ++q) {  // internal order
    bptr[q] = io[order[q]].b;
    xptr[q] = io[order[q]].x;
  }
  DevMem bdev(sizeof(void *) * npairs), xdev(sizeof(void *) * npairs);
  MDP_HIP(hipMemcpyAsync(bdev.get(), bptr.data(), sizeof(void *) * npairs, hipMemcpyHostToDevice, s));
  MDP_HIP(hipMemcpyAsync(xdev.get(), xptr.data(), sizeof(void *) * npairs, hipMemcpyHostToDevice, s));
  const int g = grid_for(n);
  double *bg = dptr<double>(W.bp), *xg = dptr<double>(W.xp);
  hipLaunchKernelGGL(gather_pairs_kernel, dim3(g), dim3(kThreads), 0, s, static_cast<int64_t>(n),
                     dptr<const int>(gpair), dptr<const int>(gidx), dptr<const double *const>(bdev), bg);
  if (use_x0)
    hipLaunchKernelGGL(gather_pairs_kernel, dim3(g), dim3(kThreads), 0, s, static_cast<int64_t>(n),
                       dptr<const int>(gpair), dptr<const int>(gidx), dptr<const double *const>(xdev), xg);
  int rc;
  std::vector<mdp_stats> sti(st ? static_cast<size_t>(npairs) : 0);  // internal order
  if (opt.precision == MDP_MIXED) {
    Problem<float> pb{&A, pc32.get(), &layout, &W, &opt, &graphs};
    rc = fgmres<float>(pb, bg, xg, use_x0, s, st ? sti.data() : nullptr);
  } else {
    Problem<double> pb{&A, pc64.get(), &layout, &W, &opt, &graphs};
    rc = fgmres<double>(pb, bg, xg, use_x0, s, st ? sti.data() : nullptr);
  }
  hipLaunchKernelGGL(scatter_pairs_kernel, dim3(g), dim3(kThreads), 0, s, static_cast<int64_t>(n),
                     dptr<const int>(gpair), dptr<const int>(gidx), static_cast<const double *>(xg),
                     dptr<double *const>(xdev), static_cast<const int *>(nullptr));
  MDP_HIP(hipGetLastError());
  MDP_HIP(hipStreamSynchronize(s));  // bdev / xdev die here
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (st)
    for (int q = 0; q < npairs; ++q) {
      const int p = order[q];
      st[p] = sti[q];
      st[p].solve_ms = ms;
      st[p].setup_ms = sys[p]->setup_ms;
    }
  return rc;
}

}  // namespace mdp
