// CPU check of the host-side sparse layouts and the Arnoldi tile plan that
// the library uploads (formats.hpp).  For every matrix of the host systems
// named on the command line it rebuilds each eligible layout and replays the
// index arithmetic of the matching kernel on the CPU: every index it would
// read must lie inside its array, and the product it would form must equal
// the CSR product.  It then checks the tile plan on those systems, on their
// concatenation and on boundary sizes.  Prints "failures: N" and exits with
// status 1 when N > 0.
#include <cmath>
#include <cstdio>
#include <vector>

#include "formats.hpp"
#include "setup.hpp"

using namespace mdp;

static int fails = 0;
#define CHECK(c, ...)                                          \
  do {                                                         \
    if (!(c)) {                                                \
      if (++fails <= 20) {                                     \
        std::printf("FAIL line %d: ", __LINE__);               \
        std::printf(__VA_ARGS__);                              \
        std::printf("\n");                                     \
      }                                                        \
    }                                                          \
  } while (0)

static std::vector<double> csr_product(const HCsr &h, const std::vector<double> &x) {
  std::vector<double> y(h.nr, 0.0);
  for (int32_t i = 0; i < h.nr; ++i)
    for (int32_t k = h.ptr[i]; k < h.ptr[i + 1]; ++k) y[i] += h.val[k] * x[h.col[k]];
  return y;
}

static void same(const char *what, const char *fmt, const std::vector<double> &y, const std::vector<double> &r) {
  double num = 0.0, den = 0.0;
  for (size_t i = 0; i < y.size(); ++i) {
    num += (y[i] - r[i]) * (y[i] - r[i]);
    den += r[i] * r[i];
  }
  CHECK(num <= 1e-24 * den + 1e-300, "%s (%s): relative error %g", what, fmt, std::sqrt(num / (den + 1e-300)));
}

// CSR with lanes or one thread per row: row i reads col[s..e) and, for
// batch entries past the row end, col[s].
static void check_csr(const char *what, const HCsr &h, const std::vector<double> &x, const std::vector<double> &r) {
  std::vector<double> y(h.nr, 0.0);
  CHECK(static_cast<int64_t>(h.ptr.size()) == h.nr + 1, "%s: row pointer size", what);
  for (int32_t i = 0; i < h.nr; ++i) {
    const int32_t s = h.ptr[i], e = h.ptr[i + 1];
    CHECK(0 <= s && s <= e && e <= h.nnz(), "%s: row %d range", what, i);
    for (int32_t p = s; p < e; ++p) {
      CHECK(h.col[p] >= 0 && h.col[p] < h.nc, "%s: row %d column %d", what, i, h.col[p]);
      if (h.col[p] >= 0 && h.col[p] < h.nc) y[i] += h.val[p] * x[h.col[p]];
    }
  }
  same(what, "csr", y, r);
}

// Sliced ELL: slice s spans soff[s]..soff[s+1], a multiple of 64; lane L
// reads entries soff[s] + L + 64 k, past the slice width col[soff[s] + L].
static void check_sell(const char *what, const HCsr &h, const SliceStats &st, const std::vector<double> &x,
                       const std::vector<double> &r) {
  const SellLayout L = sell_layout(h, st);
  std::vector<double> y(h.nr, 0.0);
  CHECK(L.nslices == (h.nr + 63) / 64, "%s: slice count", what);
  CHECK(static_cast<int64_t>(L.col.size()) == st.padded && L.val.size() == L.col.size(), "%s: sell sizes", what);
  CHECK(L.soff[L.nslices] == static_cast<int32_t>(L.col.size()), "%s: last slice offset", what);
  for (int32_t sl = 0; sl < L.nslices; ++sl) {
    const int32_t o0 = L.soff[sl], o1 = L.soff[sl + 1];
    CHECK(o0 <= o1 && (o1 - o0) % 64 == 0, "%s: slice %d offsets", what, sl);
    for (int32_t lane = 0; lane < 64; ++lane) {
      const int32_t row = sl * 64 + lane;
      if (row >= h.nr) continue;
      for (int32_t o = o0 + lane; o < o1; o += 64) {
        const int32_t c = L.col[o];
        CHECK(c >= 0 && c < h.nc, "%s: sell column %d", what, c);
        if (c >= 0 && c < h.nc) y[row] += L.val[o] * x[c];
      }
    }
  }
  same(what, "sliced ELL", y, r);
}

// Diagonals: row i reads val[d * nr + i] and x[i + offs[d]] when in range.
static void dia_part(const std::vector<int32_t> &offs, const std::vector<double> &val, const HCsr &h,
                     const std::vector<double> &x, std::vector<double> &y) {
  for (int32_t i = 0; i < h.nr; ++i)
    for (size_t d = 0; d < offs.size(); ++d) {
      const int64_t c = static_cast<int64_t>(i) + offs[d];
      if (c >= 0 && c < h.nc) y[i] += val[d * h.nr + i] * x[c];
    }
}

static void check_dia(const char *what, const HCsr &h, const std::vector<int32_t> &offs,
                      const std::vector<double> &x, const std::vector<double> &r) {
  const DiaLayout L = dia_layout(h, offs);
  CHECK(L.val.size() == offs.size() * static_cast<size_t>(h.nr), "%s: dia size", what);
  CHECK(std::is_sorted(L.offs.begin(), L.offs.end()) && L.offs.size() <= static_cast<size_t>(kMaxDiag),
        "%s: offsets", what);
  std::vector<double> y(h.nr, 0.0);
  dia_part(L.offs, L.val, h, x, y);
  same(what, "diagonal", y, r);
}

static void check_hyb(const char *what, const HCsr &h, const std::vector<int32_t> &offs,
                      const std::vector<double> &x, const std::vector<double> &r) {
  const HybLayout L = hyb_layout(h, offs);
  CHECK(L.dval.size() == offs.size() * static_cast<size_t>(h.nr), "%s: hyb diagonal size", what);
  CHECK(static_cast<int64_t>(L.ptr.size()) == h.nr + 1 && L.ptr[h.nr] == static_cast<int32_t>(L.col.size()),
        "%s: hyb remainder pointers", what);
  std::vector<double> y(h.nr, 0.0);
  dia_part(L.offs, L.dval, h, x, y);
  for (int32_t i = 0; i < h.nr; ++i)
    for (int32_t p = L.ptr[i]; p < L.ptr[i + 1]; ++p) {
      const int32_t c = L.col[p];
      CHECK(c >= 0 && c < h.nc, "%s: remainder column %d", what, c);
      CHECK(std::find(L.offs.begin(), L.offs.end(), c - i) == L.offs.end(), "%s: remainder entry on a diagonal",
            what);
      if (c >= 0 && c < h.nc) y[i] += L.val[p] * x[c];
    }
  same(what, "diagonals + remainder", y, r);
  // the rows dispatched first are exactly the trailing run of rows that all
  // have remainder entries (none when every row has some)
  CHECK(L.split >= 1 && L.split <= h.nr, "%s: hyb split %d", what, L.split);
  int32_t run = h.nr;
  while (run > 0 && L.ptr[run] > L.ptr[run - 1]) --run;
  CHECK(L.split == (run == 0 ? h.nr : run), "%s: hyb split %d, trailing run from %d", what, L.split, run);
  std::printf("%-12s hyb split=%d of %d\n", what, L.split, h.nr);
}

static void check_matrix(const char *what, const HCsr &h) {
  if (h.nr == 0) return;
  std::vector<double> x(h.nc);
  for (int32_t j = 0; j < h.nc; ++j) x[j] = std::sin(0.37 * j + 1.0) + 0.01 * (j % 7);
  const std::vector<double> r = csr_product(h, x);
  const SliceStats st = slice_stats(h);
  const std::vector<int32_t> offs = dia_offsets(h);
  const std::vector<int32_t> hoffs = offs.empty() ? hyb_offsets(h) : std::vector<int32_t>{};
  check_csr(what, h, x, r);
  if (sell_possible(st, h.nnz(), 2.0)) check_sell(what, h, st, x, r);
  if (!offs.empty()) check_dia(what, h, offs, x, r);
  if (!hoffs.empty()) check_hyb(what, h, hoffs, x, r);
  std::printf("%-12s nr=%8d nnz=%9lld sell=%d dia=%zu hyb=%zu\n", what, h.nr, static_cast<long long>(h.nnz()),
              static_cast<int>(sell_possible(st, h.nnz(), 2.0)), offs.size(), hoffs.size());
}

// The plan covers every range exactly, tile by tile in order, with lengths
// in [1, kTileElems] differing by at most one inside a range; pairs own
// consecutive tiles; a long vector gets a multiple of the 256 compute units.
static void check_tiles(const char *what, const std::vector<std::vector<std::pair<int64_t, int64_t>>> &ranges) {
  std::vector<int32_t> off;
  const std::vector<Tile> tl = plan_tiles(ranges, off);
  CHECK(off.size() == ranges.size() + 1 && off.front() == 0 && off.back() == static_cast<int32_t>(tl.size()),
        "%s: tile offsets", what);
  int64_t total = 0;
  size_t nonempty = 0;
  for (size_t p = 0; p < ranges.size(); ++p) {
    size_t t = off[p];
    for (const auto &r : ranges[p]) {
      total += r.second;
      if (r.second == 0) continue;
      ++nonempty;
      int64_t at = r.first;
      int32_t lo = kTileElems, hi = 0;
      while (at < r.first + r.second && t < static_cast<size_t>(off[p + 1])) {
        CHECK(tl[t].start == at && tl[t].pair == static_cast<int32_t>(p), "%s: tile %zu start/pair", what, t);
        CHECK(tl[t].len >= 1 && tl[t].len <= kTileElems, "%s: tile %zu length %d", what, t, tl[t].len);
        lo = std::min(lo, tl[t].len);
        hi = std::max(hi, tl[t].len);
        at += tl[t].len;
        ++t;
      }
      CHECK(at == r.first + r.second, "%s: pair %zu range not covered", what, p);
      CHECK(hi - lo <= 1, "%s: pair %zu tile lengths %d..%d", what, p, lo, hi);
    }
    CHECK(t == static_cast<size_t>(off[p + 1]), "%s: pair %zu has extra tiles", what, p);
  }
  const int64_t target = tile_target(total);
  CHECK(static_cast<int64_t>(tl.size()) >= target, "%s: %zu tiles below the target %lld", what, tl.size(),
        static_cast<long long>(target));
  if (nonempty == 1 && total >= kCus * kTileElems)
    CHECK(tl.size() % kCus == 0, "%s: %zu tiles is not a multiple of %lld", what, tl.size(),
          static_cast<long long>(kCus));
  std::printf("tiles %-28s n=%10lld tiles=%7zu target=%7lld\n", what, static_cast<long long>(total), tl.size(),
              static_cast<long long>(target));
}

// A level's fused restriction restricts b to what R restricts the residual
// of the first smoothing iterate to: Rf b = R (b - A D^-1 b), D the l1 norms.
static int fused_levels = 0;
static void check_fused(const char *what, const HLevel &L) {
  if (L.Rf.nr == 0) return;
  ++fused_levels;
  const int32_t n = L.A.nr;
  CHECK(L.Rf.nr == L.R.nr && L.Rf.nc == n, "%s: fused restriction shape", what);
  std::vector<double> b(n), t(n), r(n), y1(L.R.nr, 0.0), y2(L.R.nr, 0.0);
  for (int32_t i = 0; i < n; ++i) {
    b[i] = std::cos(0.91 * i + 0.3) + 0.05 * (i % 11);
    t[i] = b[i] / L.dl1[i];
  }
  for (int32_t i = 0; i < n; ++i) {
    double a = 0.0;
    for (int32_t p = L.A.ptr[i]; p < L.A.ptr[i + 1]; ++p) a += L.A.val[p] * t[L.A.col[p]];
    r[i] = b[i] - a;
  }
  double scale = 0.0;
  for (int32_t i = 0; i < L.R.nr; ++i) {
    for (int32_t p = L.Rf.ptr[i]; p < L.Rf.ptr[i + 1]; ++p) y1[i] += L.Rf.val[p] * b[L.Rf.col[p]];
    for (int32_t p = L.R.ptr[i]; p < L.R.ptr[i + 1]; ++p) y2[i] += L.R.val[p] * r[L.R.col[p]];
    scale = std::max(scale, std::fabs(y2[i]));
  }
  double err = 0.0;
  for (int32_t i = 0; i < L.R.nr; ++i) err = std::max(err, std::fabs(y1[i] - y2[i]));
  CHECK(err <= 1e-12 * std::max(scale, 1.0), "%s: fused restriction differs by %.3g (scale %.3g)", what, err, scale);
  std::printf("%-12s fused restriction nnz=%lld (R %lld, A %lld)\n", what, static_cast<long long>(L.Rf.nnz()),
              static_cast<long long>(L.R.nnz()), static_cast<long long>(L.A.nnz()));
}

int main(int argc, char **argv) {
  std::vector<std::vector<std::pair<int64_t, int64_t>>> batch;
  int64_t at = 0;
  for (int a = 1; a < argc; ++a) {
    HostSystem s;
    mdp_options o{};
    load_host_system(argv[a], s, o);
    std::printf("== %s: n=%d n_o=%d n_g=%d\n", argv[a], s.n, s.n_o, s.n_g);
    check_matrix("A", s.A);
    check_matrix("A_GO", s.Ago);
    check_matrix("A_OG", s.Aog);
    char name[32];
    for (size_t l = 0; l < s.Ho.lv.size(); ++l) {
      std::snprintf(name, sizeof name, "S[%zu].A", l);
      check_matrix(name, s.Ho.lv[l].A);
      std::snprintf(name, sizeof name, "S[%zu].P", l);
      check_matrix(name, s.Ho.lv[l].P);
      std::snprintf(name, sizeof name, "S[%zu].R", l);
      check_matrix(name, s.Ho.lv[l].R);
      check_fused(name, s.Ho.lv[l]);
    }
    for (size_t l = 0; l < s.Hg.lv.size(); ++l) {
      std::snprintf(name, sizeof name, "G[%zu].A", l);
      check_matrix(name, s.Hg.lv[l].A);
      std::snprintf(name, sizeof name, "G[%zu].P", l);
      check_matrix(name, s.Hg.lv[l].P);
      std::snprintf(name, sizeof name, "G[%zu].R", l);
      check_matrix(name, s.Hg.lv[l].R);
      check_fused(name, s.Hg.lv[l]);
    }
    check_tiles("one system", {{{0, s.n_o}, {s.n_o, s.n_g}}});
    batch.push_back({{at, s.n_o}, {at + s.n_o, s.n_g}});
    at += s.n;
  }
  if (!batch.empty()) check_tiles("all systems as a batch", batch);
  const int64_t full = kCus * kTileElems;
  for (int64_t n : {int64_t{1}, int64_t{63}, int64_t{64}, int64_t{65}, int64_t{1000}, full - 1, full, full + 1,
                    int64_t{1090000}, int64_t{4326400}}) {
    char name[48];
    std::snprintf(name, sizeof name, "one range of %lld", static_cast<long long>(n));
    check_tiles(name, {{{0, n}}});
  }
  std::vector<std::vector<std::pair<int64_t, int64_t>>> tiny;
  for (int p = 0; p < 1000; ++p) tiny.push_back({{p * 7, 5}, {p * 7 + 5, p % 3}});
  check_tiles("1000 small pairs", tiny);
  std::printf("fused restrictions: %d\n", fused_levels);
  std::printf("failures: %d\n", fails);
  return fails ? 1 : 0;
}
