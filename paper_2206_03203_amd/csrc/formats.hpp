// Host-side rules and layouts of the device sparse formats, and the tile
// plan of the Arnoldi passes.  Plain C++ (no device code): the library builds
// these arrays at set-up and uploads them; the CPU tests check them against
// the kernels' indexing.
#pragma once

#include <algorithm>
#include <cstdint>
#include <iterator>
#include <limits>
#include <unordered_map>
#include <utility>
#include <vector>

#include "host_csr.hpp"
#include "types.hpp"

namespace mdp {

// Lanes per row for the CSR-vector kernel: enough that one batch of
// kCsrBatch entries per lane covers an average row.
inline int choose_lpr(int64_t nnz, int32_t nr) {
  const double avg = nr > 0 ? static_cast<double>(nnz) / nr : 0.0;
  int l = 4;
  while (l * kCsrBatch < avg && l < 64) l *= 2;
  return l;
}

struct FormatChoice {
  bool sell = false;
  bool scalar = false;
  int lpr = 8;
  int batch = kCsrBatch;  // CSR-vector entries in flight per lane (4 or 8)
  bool dia = false;
  bool hyb = false;
};

struct SliceStats {
  int64_t padded = 0;  // entries of the sliced-ELL layout (64-row slices)
  int32_t maxlen = 0;
};

inline SliceStats slice_stats(const HCsr &h) {
  SliceStats st;
  const int32_t ns = (h.nr + 63) / 64;
  for (int32_t sl = 0; sl < ns; ++sl) {
    int32_t w = 0;
    for (int32_t r = sl * 64; r < std::min(h.nr, sl * 64 + 64); ++r) w = std::max(w, h.ptr[r + 1] - h.ptr[r]);
    st.padded += 64 * static_cast<int64_t>(w);
    st.maxlen = std::max(st.maxlen, w);
  }
  return st;
}

inline bool sell_possible(const SliceStats &st, int64_t nnz, double max_padding) {
  return st.maxlen <= 64 && static_cast<double>(st.padded) <= max_padding * static_cast<double>(std::max<int64_t>(nnz, 1)) &&
         st.padded < std::numeric_limits<int32_t>::max();
}

// The distinct diagonal offsets (column - row) of a matrix, ascending, when
// there are at most kMaxDiag of them and the diagonal layout pads the
// entries by at most 20%; empty otherwise.
inline std::vector<int32_t> dia_offsets(const HCsr &h) {
  // each chunk of rows collects its offsets (giving up past kMaxDiag), then
  // the chunks' sets are merged
  const int T = setup_workers();
  std::vector<std::vector<int32_t>> part(static_cast<size_t>(T));
  std::vector<char> over(static_cast<size_t>(T), 0);
  parallel_chunks(h.nr, [&](int64_t b, int64_t e, int t) {
    std::vector<int32_t> &offs = part[t];
    for (int64_t i = b; i < e && !over[t]; ++i)
      for (int32_t k = h.ptr[i]; k < h.ptr[i + 1]; ++k) {
        const int32_t d = h.col[k] - static_cast<int32_t>(i);
        const auto it = std::lower_bound(offs.begin(), offs.end(), d);
        if (it != offs.end() && *it == d) continue;
        if (static_cast<int>(offs.size()) == kMaxDiag) {
          over[t] = 1;
          break;
        }
        offs.insert(it, d);
      }
  });
  std::vector<int32_t> offs;
  for (int t = 0; t < T; ++t) {
    if (over[t]) return {};
    std::vector<int32_t> m;
    std::set_union(offs.begin(), offs.end(), part[t].begin(), part[t].end(), std::back_inserter(m));
    if (static_cast<int>(m.size()) > kMaxDiag) return {};
    offs.swap(m);
  }
  if (static_cast<double>(offs.size()) * h.nr > 1.2 * static_cast<double>(std::max<int64_t>(h.nnz(), 1))) return {};
  return offs;
}

// Diagonals for the diagonals-plus-remainder layout: the offsets that hold
// an entry in at least half of the rows (at most kMaxDiag, the fullest), when
// together they hold at least 80% of the entries with at most 25% padding;
// empty otherwise.  Rows of more than kMaxDiag + 4 entries on average are
// not looked at.
inline std::vector<int32_t> hyb_offsets(const HCsr &h) {
  if (h.nr == 0 || h.nnz() > static_cast<int64_t>(kMaxDiag + 4) * h.nr) return {};
  const int T = setup_workers();
  std::vector<std::unordered_map<int32_t, int64_t>> part(static_cast<size_t>(T));
  parallel_chunks(h.nr, [&](int64_t b, int64_t e, int t) {
    auto &c = part[t];
    c.reserve(64);
    for (int64_t i = b; i < e; ++i)
      for (int32_t k = h.ptr[i]; k < h.ptr[i + 1]; ++k) ++c[h.col[k] - static_cast<int32_t>(i)];
  });
  std::unordered_map<int32_t, int64_t> count;
  for (const auto &c : part)
    for (const auto &kv : c) count[kv.first] += kv.second;
  std::vector<std::pair<int64_t, int32_t>> full;
  for (const auto &c : count)
    if (2 * c.second >= h.nr) full.emplace_back(c.second, c.first);
  std::sort(full.begin(), full.end(), [](const auto &a, const auto &b) {
    return a.first != b.first ? a.first > b.first : a.second < b.second;
  });
  if (full.size() > static_cast<size_t>(kMaxDiag)) full.resize(kMaxDiag);
  int64_t covered = 0;
  std::vector<int32_t> offs;
  for (const auto &f : full) {
    covered += f.first;
    offs.push_back(f.second);
  }
  std::sort(offs.begin(), offs.end());
  const double stored = static_cast<double>(offs.size()) * h.nr;
  if (offs.empty() || covered < 0.8 * h.nnz() || stored > 1.25 * covered) return {};
  return offs;
}

// Fixed rule (also the autotuner's fallback): diagonal storage for stencil
// matrices, diagonals plus a remainder for stencils with a few irregular
// couplings, sliced ELL when the slices carry at most 15% padding, one
// thread per row for other short rows, else enough lanes per row for
// kCsrBatch entries each.
inline FormatChoice heuristic_format(const HCsr &h, const SliceStats &st, bool dia_ok, bool hyb_ok) {
  FormatChoice f;
  if (dia_ok) {
    f.dia = true;
    return f;
  }
  if (hyb_ok) {
    f.hyb = true;
    return f;
  }
  const int64_t nnz = h.nnz();
  f.lpr = choose_lpr(nnz, h.nr);
  f.sell = h.nr > 0 && sell_possible(st, nnz, 1.15);
  f.scalar = !f.sell && (h.nr > 0 ? static_cast<double>(nnz) / h.nr : 0.0) <= 12.0;
  return f;
}

// Sliced ELL: 64-row slices, entry k of the row at lane L of slice s at
// soff[s] + 64 k + L.  A slice is as wide as its longest row; padding entries
// carry value 0 and a valid column of the slice (the lane's last one, or the
// slice's first).
struct SellLayout {
  int32_t nslices = 0;
  std::vector<int32_t> soff, col;
  std::vector<double> val;
};

inline SellLayout sell_layout(const HCsr &h, const SliceStats &st) {
  SellLayout L;
  const int32_t ns = (h.nr + 63) / 64;
  L.nslices = ns;
  L.soff.assign(static_cast<size_t>(ns) + 1, 0);
  for (int32_t sl = 0; sl < ns; ++sl) {
    int32_t w = 0;
    for (int32_t r = sl * 64; r < std::min(h.nr, sl * 64 + 64); ++r) w = std::max(w, h.ptr[r + 1] - h.ptr[r]);
    L.soff[sl + 1] = L.soff[sl] + w * 64;
  }
  L.col.assign(static_cast<size_t>(st.padded), 0);
  L.val.assign(static_cast<size_t>(st.padded), 0.0);
  parallel_chunks(ns, [&](int64_t sb, int64_t se, int) {
    for (int64_t sl = sb; sl < se; ++sl) {
      const int32_t r0 = static_cast<int32_t>(sl) * 64, r1 = std::min(h.nr, r0 + 64);
      const int64_t o = L.soff[sl];
      const int32_t w = static_cast<int32_t>((L.soff[sl + 1] - o) / 64);
      int32_t first = 0;
      for (int32_t r = r1 - 1; r >= r0; --r)
        if (h.ptr[r + 1] > h.ptr[r]) first = h.col[h.ptr[r]];
      for (int32_t lane = 0; lane < 64; ++lane) {
        const int32_t r = r0 + lane;
        const int32_t len = r < r1 ? h.ptr[r + 1] - h.ptr[r] : 0;
        int32_t lastc = first;
        for (int32_t k = 0; k < w; ++k) {
          const int64_t dst = o + static_cast<int64_t>(k) * 64 + lane;
          if (k < len) {
            lastc = h.col[h.ptr[r] + k];
            L.val[dst] = h.val[h.ptr[r] + k];
          }
          L.col[dst] = lastc;
        }
      }
    }
  });
  return L;
}

// Diagonal storage: entry (i, i + offs[d]) at val[d * nr + i], zero where
// absent.
struct DiaLayout {
  std::vector<int32_t> offs;
  std::vector<double> val;
};

inline DiaLayout dia_layout(const HCsr &h, const std::vector<int32_t> &offs) {
  DiaLayout L;
  L.offs = offs;
  L.val.assign(offs.size() * static_cast<size_t>(h.nr), 0.0);
  parallel_chunks(h.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i)
      for (int32_t k = h.ptr[i]; k < h.ptr[i + 1]; ++k) {
        const size_t di = std::lower_bound(offs.begin(), offs.end(), h.col[k] - static_cast<int32_t>(i)) - offs.begin();
        L.val[di * h.nr + i] = h.val[k];
      }
  });
  return L;
}

// Diagonals plus a CSR remainder: the entries on the offsets `offs` in
// diagonal storage (dval, as above), every other entry in the CSR ptr / col /
// val, in row order.
// split: first row of the trailing run of rows that all have remainder
// entries (nr when the last row has none, or when every row has some).  In a
// two-block system these are the fracture rows, whose remainder entries gather
// from far-away columns; the product dispatches them first.
struct HybLayout {
  std::vector<int32_t> offs, ptr, col;
  std::vector<double> dval, val;
  int32_t split = 0;
};

inline HybLayout hyb_layout(const HCsr &h, const std::vector<int32_t> &offs) {
  HybLayout L;
  L.offs = offs;
  L.dval.assign(offs.size() * static_cast<size_t>(h.nr), 0.0);
  L.ptr.assign(static_cast<size_t>(h.nr) + 1, 0);
  // first pass: the diagonal entries and the remainder's row lengths; second
  // pass: the remainder at its row offsets
  auto on_diag = [&](int32_t i, int32_t k) {
    const int32_t off = h.col[k] - i;
    const auto it = std::lower_bound(offs.begin(), offs.end(), off);
    return it != offs.end() && *it == off ? static_cast<int64_t>(it - offs.begin()) : int64_t{-1};
  };
  parallel_chunks(h.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      int32_t rem = 0;
      for (int32_t k = h.ptr[i]; k < h.ptr[i + 1]; ++k) {
        const int64_t d = on_diag(static_cast<int32_t>(i), k);
        if (d >= 0)
          L.dval[static_cast<size_t>(d) * h.nr + i] = h.val[k];
        else
          ++rem;
      }
      L.ptr[i + 1] = rem;
    }
  });
  for (int32_t i = 0; i < h.nr; ++i) L.ptr[i + 1] += L.ptr[i];
  L.col.resize(static_cast<size_t>(L.ptr[h.nr]));
  L.val.resize(static_cast<size_t>(L.ptr[h.nr]));
  parallel_chunks(h.nr, [&](int64_t b, int64_t e, int) {
    for (int64_t i = b; i < e; ++i) {
      int32_t q = L.ptr[i];
      for (int32_t k = h.ptr[i]; k < h.ptr[i + 1]; ++k)
        if (on_diag(static_cast<int32_t>(i), k) < 0) {
          L.col[q] = h.col[k];
          L.val[q] = h.val[k];
          ++q;
        }
    }
  });
  L.split = h.nr;
  while (L.split > 0 && L.ptr[L.split] > L.ptr[L.split - 1]) --L.split;
  if (L.split == 0) L.split = h.nr;
  return L;
}

// Tiles.  Each Arnoldi pass gives one workgroup per tile and every tile the
// same work, so the tile count is a multiple of the 256 compute units when
// the vectors are long enough (a partly filled last round of workgroups costs
// as much as a full one), with at most kTileElems entries per tile and, for
// short vectors, at least kMinTile.  The tiles are shared among the ranges in
// proportion to their lengths (largest remainders first); each range is cut
// into tiles whose lengths differ by at most one.
constexpr int64_t kCus = 256;
constexpr int64_t kMinTile = 64;

inline int64_t tile_target(int64_t n) {
  const int64_t fewest = (n + kTileElems - 1) / kTileElems;
  const int64_t most = std::max<int64_t>(1, (n + kMinTile - 1) / kMinTile);
  const int64_t balanced = (fewest + kCus - 1) / kCus * kCus;
  return std::min(balanced, std::max(fewest, most));
}

// ranges[p] = the (start, length) pieces of pair p in the global vector.
// Returns the tiles grouped by pair; tile_off[p] .. tile_off[p + 1] are pair
// p's tiles.
inline std::vector<Tile> plan_tiles(const std::vector<std::vector<std::pair<int64_t, int64_t>>> &ranges,
                                    std::vector<int32_t> &tile_off) {
  const int npairs = static_cast<int>(ranges.size());
  struct Share {
    int p;
    int64_t start, len, k;
    double rem;
  };
  std::vector<Share> sh;
  int64_t total = 0;
  for (int p = 0; p < npairs; ++p)
    for (const auto &r : ranges[p]) {
      total += r.second;
      if (r.second > 0) sh.push_back(Share{p, r.first, r.second, 0, 0.0});
    }
  const int64_t target = tile_target(total);
  int64_t given = 0;
  for (Share &x : sh) {
    const double exact = static_cast<double>(x.len) * target / std::max<int64_t>(total, 1);
    x.k = static_cast<int64_t>(exact);
    x.rem = exact - x.k;
    given += x.k;
  }
  std::vector<size_t> by_rem(sh.size());
  for (size_t i = 0; i < sh.size(); ++i) by_rem[i] = i;
  std::stable_sort(by_rem.begin(), by_rem.end(), [&](size_t a, size_t b) { return sh[a].rem > sh[b].rem; });
  for (size_t i = 0; i < by_rem.size() && given < target; ++i, ++given) ++sh[by_rem[i]].k;
  std::vector<Tile> tl;
  tile_off.assign(static_cast<size_t>(npairs) + 1, 0);
  size_t q = 0;
  for (int p = 0; p < npairs; ++p) {
    for (; q < sh.size() && sh[q].p == p; ++q) {
      Share &x = sh[q];
      x.k = std::min(x.len, std::max({x.k, int64_t{1}, (x.len + kTileElems - 1) / kTileElems}));
      for (int64_t i = 0; i < x.k; ++i) {
        const int64_t lo = i * x.len / x.k, hi = (i + 1) * x.len / x.k;
        tl.push_back(Tile{x.start + lo, static_cast<int32_t>(hi - lo), p});
      }
    }
    tile_off[p + 1] = static_cast<int32_t>(tl.size());
  }
  return tl;
}

}  // namespace mdp
