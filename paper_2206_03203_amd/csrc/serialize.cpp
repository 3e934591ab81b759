// Hierarchy files: the complete host setup of a handle (the [Omega; Gamma]
// permutation, the blocks of eq. (4), S~ of eq. (7) and both SA-AMG
// hierarchies of Section 3.3) written to a file and read back, so that a
// system can be solved again without repeating its setup.
//
// Layout (little-endian): the 8-byte tag "MDPHIER1", a format version, the
// AMG options the hierarchy was built with, the sizes and permutation, six
// CSR matrices, the two hierarchies (version 2: each level with its fused
// restriction, 0 x 0 when unused; version 1, still read: without it), and a
// 64-bit FNV-1a checksum of every byte before it.  Reading checks the tag,
// version, checksum, every length against the bytes left, and the structure
// of every matrix, and reports any failure as MDP_EINVAL without touching the
// output.
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>

#include "setup.hpp"

namespace mdp {

namespace {

constexpr char kTag[8] = {'M', 'D', 'P', 'H', 'I', 'E', 'R', '1'};
constexpr uint32_t kVersion = 2;  // 2 adds each level's fused restriction; 1 is still read

uint64_t fnv1a(const unsigned char *p, size_t n) {
  uint64_t h = 1469598103934665603ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

struct Writer {
  std::vector<unsigned char> buf;
  void raw(const void *p, size_t n) {
    const auto *c = static_cast<const unsigned char *>(p);
    buf.insert(buf.end(), c, c + n);
  }
  template <typename T>
  void pod(T v) {
    raw(&v, sizeof(T));
  }
  template <typename T>
  void vec(const std::vector<T> &v) {
    pod<int64_t>(static_cast<int64_t>(v.size()));
    if (!v.empty()) raw(v.data(), v.size() * sizeof(T));
  }
  void csr(const HCsr &m) {
    pod<int32_t>(m.nr);
    pod<int32_t>(m.nc);
    vec(m.ptr);
    vec(m.col);
    vec(m.val);
  }
  void hier(const HHier &h) {
    pod<int32_t>(static_cast<int32_t>(h.lv.size()));
    pod<uint8_t>(h.dense ? 1 : 0);
    vec(h.coarse_inv);
    for (const HLevel &l : h.lv) {
      csr(l.A);
      csr(l.P);
      csr(l.R);
      csr(l.Rf);
      vec(l.dl1);
      vec(l.agg);
    }
  }
};

struct Bad {};  // any malformed input

struct Reader {
  const unsigned char *p;
  size_t left;
  uint32_t version = kVersion;
  void raw(void *dst, size_t n) {
    if (n > left) throw Bad{};
    std::memcpy(dst, p, n);
    p += n;
    left -= n;
  }
  template <typename T>
  T pod() {
    T v;
    raw(&v, sizeof(T));
    return v;
  }
  template <typename T>
  std::vector<T> vec() {
    const int64_t n = pod<int64_t>();
    if (n < 0 || static_cast<uint64_t>(n) > left / sizeof(T)) throw Bad{};
    std::vector<T> v(static_cast<size_t>(n));
    if (n > 0) raw(v.data(), static_cast<size_t>(n) * sizeof(T));
    return v;
  }
  HCsr csr() {
    HCsr m;
    m.nr = pod<int32_t>();
    m.nc = pod<int32_t>();
    m.ptr = vec<int32_t>();
    m.col = vec<int32_t>();
    m.val = vec<double>();
    if (m.nr < 0 || m.nc < 0 || m.ptr.size() != static_cast<size_t>(m.nr) + 1 || m.ptr[0] != 0 ||
        static_cast<size_t>(m.ptr[m.nr]) != m.col.size() || m.col.size() != m.val.size())
      throw Bad{};
    for (int32_t i = 0; i < m.nr; ++i)
      if (m.ptr[i + 1] < m.ptr[i]) throw Bad{};
    for (int32_t c : m.col)
      if (c < 0 || c >= m.nc) throw Bad{};
    return m;
  }
  HHier hier() {
    HHier h;
    const int32_t nl = pod<int32_t>();
    if (nl < 0 || nl > 64) throw Bad{};
    h.dense = pod<uint8_t>() != 0;
    h.coarse_inv = vec<double>();
    h.lv.resize(static_cast<size_t>(nl));
    for (HLevel &l : h.lv) {
      l.A = csr();
      l.P = csr();
      l.R = csr();
      l.Rf = version >= 2 ? csr() : HCsr::empty(0, 0);
      l.dl1 = vec<double>();
      l.agg = vec<int32_t>();
    }
    // consistency between levels: square operators, P from level l+1 to l
    for (int32_t k = 0; k < nl; ++k) {
      const HLevel &l = h.lv[k];
      if (l.A.nr != l.A.nc || l.dl1.size() != static_cast<size_t>(l.A.nr)) throw Bad{};
      if (k + 1 < nl) {
        const int32_t nc = h.lv[k + 1].A.nr;
        if (l.P.nr != l.A.nr || l.P.nc != nc || l.R.nr != nc || l.R.nc != l.A.nr) throw Bad{};
        if (l.Rf.nr != 0 && (l.Rf.nr != nc || l.Rf.nc != l.A.nr)) throw Bad{};
        if (l.agg.size() != static_cast<size_t>(l.A.nr)) throw Bad{};
        for (int32_t a : l.agg)
          if (a < -1 || a >= nc) throw Bad{};
      } else if (!l.agg.empty() || l.Rf.nr != 0) {
        throw Bad{};
      }
    }
    if (h.dense) {
      const int64_t nc = nl > 0 ? h.lv.back().A.nr : 0;
      if (static_cast<int64_t>(h.coarse_inv.size()) != nc * nc) throw Bad{};
    }
    return h;
  }
};

}  // namespace

void save_host_system(const HostSystem &s, const mdp_options &o, const char *path) {
  Writer w;
  w.raw(kTag, sizeof(kTag));
  w.pod<uint32_t>(kVersion);
  w.pod<double>(o.strength_theta);
  w.pod<int32_t>(o.max_coarse);
  w.pod<int32_t>(o.max_dense);
  w.pod<int32_t>(o.max_levels);
  w.pod<int32_t>(s.n);
  w.pod<int32_t>(s.n_o);
  w.pod<int32_t>(s.n_g);
  w.pod<uint8_t>(s.identity ? 1 : 0);
  w.pod<uint8_t>(s.symmetric ? 1 : 0);
  w.vec(s.perm);
  for (const HCsr *m : {&s.A, &s.Aoo, &s.Aog, &s.Ago, &s.Agg, &s.S}) w.csr(*m);
  w.hier(s.Ho);
  w.hier(s.Hg);
  const uint64_t sum = fnv1a(w.buf.data(), w.buf.size());
  w.pod<uint64_t>(sum);
  std::unique_ptr<FILE, int (*)(FILE *)> f(std::fopen(path, "wb"), &std::fclose);
  if (!f) throw SetupError{MDP_EINVAL, std::string("cannot open ") + path + " for writing"};
  if (std::fwrite(w.buf.data(), 1, w.buf.size(), f.get()) != w.buf.size())
    throw SetupError{MDP_EINVAL, std::string("short write to ") + path};
  if (std::fflush(f.get()) != 0) throw SetupError{MDP_EINVAL, std::string("cannot write ") + path};
}

void load_host_system(const char *path, HostSystem &out, mdp_options &amg) {
  std::unique_ptr<FILE, int (*)(FILE *)> f(std::fopen(path, "rb"), &std::fclose);
  if (!f) throw SetupError{MDP_EINVAL, std::string("cannot open ") + path};
  std::vector<unsigned char> buf;
  unsigned char chunk[1 << 16];
  size_t got;
  while ((got = std::fread(chunk, 1, sizeof(chunk), f.get())) > 0) buf.insert(buf.end(), chunk, chunk + got);
  const std::string bad = std::string(path) + " is not a valid hierarchy file";
  if (buf.size() < sizeof(kTag) + sizeof(uint64_t) || std::memcmp(buf.data(), kTag, sizeof(kTag)) != 0)
    throw SetupError{MDP_EINVAL, bad};
  uint64_t stored;
  std::memcpy(&stored, buf.data() + buf.size() - sizeof(uint64_t), sizeof(uint64_t));
  if (fnv1a(buf.data(), buf.size() - sizeof(uint64_t)) != stored)
    throw SetupError{MDP_EINVAL, bad + " (checksum mismatch)"};
  Reader r{buf.data() + sizeof(kTag), buf.size() - sizeof(kTag) - sizeof(uint64_t)};
  try {
    r.version = r.pod<uint32_t>();
    if (r.version != 1 && r.version != kVersion) throw Bad{};
    amg.strength_theta = r.pod<double>();
    amg.max_coarse = r.pod<int32_t>();
    amg.max_dense = r.pod<int32_t>();
    amg.max_levels = r.pod<int32_t>();
    HostSystem s;
    s.n = r.pod<int32_t>();
    s.n_o = r.pod<int32_t>();
    s.n_g = r.pod<int32_t>();
    s.identity = r.pod<uint8_t>() != 0;
    s.symmetric = r.pod<uint8_t>() != 0;
    s.perm = r.vec<int32_t>();
    for (HCsr *m : {&s.A, &s.Aoo, &s.Aog, &s.Ago, &s.Agg, &s.S}) *m = r.csr();
    s.Ho = r.hier();
    s.Hg = r.hier();
    if (r.left != 0) throw Bad{};
    // the sizes of eq. (4) must agree with every block
    const int32_t n = s.n, no = s.n_o, ng = s.n_g;
    if (n <= 0 || no < 0 || ng < 0 || no + ng != n || s.perm.size() != static_cast<size_t>(n)) throw Bad{};
    std::vector<char> seen(static_cast<size_t>(n), 0);
    for (int32_t i = 0; i < n; ++i) {
      const int32_t v = s.perm[i];
      if (v < 0 || v >= n || seen[v] || (s.identity && v != i)) throw Bad{};
      seen[v] = 1;
    }
    if (s.A.nr != n || s.A.nc != n || s.Aoo.nr != no || s.Aoo.nc != no || s.Aog.nr != no || s.Aog.nc != ng ||
        s.Ago.nr != ng || s.Ago.nc != no || s.Agg.nr != ng || s.Agg.nc != ng || s.S.nr != no || s.S.nc != no)
      throw Bad{};
    if (s.Ho.n() != no || s.Hg.n() != ng || (no > 0 && s.Ho.lv.empty()) || (ng > 0 && s.Hg.lv.empty())) throw Bad{};
    out = std::move(s);
  } catch (const Bad &) {
    throw SetupError{MDP_EINVAL, bad};
  }
}

}  // namespace mdp
