// C ABI entry points (include/mdp.h): argument checking, error translation
// and handle lifecycle around the host setup and the device solver.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cmath>
#include <memory>
#include <mutex>
#include <new>
#include <string>

#include "dev_spgemm.hpp"
#include "ktimer.hpp"
#include "mdp.h"
#include "solver.hpp"

namespace mdp {

namespace {

// The set-up's large sparse products on the device while alive (this
// thread): those of at least MDP_DEVICE_PRODUCT_TERMS terms (default 2^22).
constexpr int64_t kDeviceProductTerms = int64_t{1} << 22;
struct DeviceProducts {
  ProductHook saved;
  DeviceProducts(bool on, void *stream) : saved(product_hook()) {
    const char *e = std::getenv("MDP_DEVICE_PRODUCT_TERMS");
    const int64_t min_terms = e ? std::max<int64_t>(1, std::atoll(e)) : kDeviceProductTerms;
    if (on) product_hook() = ProductHook{&device_spgemm, stream, min_terms};
  }
  ~DeviceProducts() { product_hook() = saved; }
  DeviceProducts(const DeviceProducts &) = delete;
  DeviceProducts &operator=(const DeviceProducts &) = delete;
};

thread_local std::string g_last_error;
std::mutex g_hook_mu;
AllocHook g_hook;

// The most recent batch plan: block-diagonal concatenations of the pairs of
// the last mdp_solve_batch call, split into chunks of bounded size.  Reused
// while the same handles, right-hand-side counts and chunk bound come back.
struct BatchCache {
  std::vector<const mdp_handle *> handles;
  std::vector<int32_t> nrhs;
  int64_t cap = 0;
  Workspace shared;  // Krylov workspace sized for the largest chunk (chunks run one after another)
  std::vector<std::unique_ptr<Batch>> chunks;
  std::vector<int> first_pair;  // per chunk
};
std::mutex g_batch_mu;
std::unique_ptr<BatchCache> g_batch;

// Device memory of mdp_apply_noalloc: the FP32 copies of its input and
// output in mixed precision.  Every GPU the library runs on holds its own
// copy, for the life of the process; kernels reach it through the address
// that hipGetSymbolAddress returns on that device (the array's name in host
// code is not a device address).
constexpr size_t kScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};  // per device, under g_scratch_mu

// The current device's address of `scratch`, looked up on the first call on
// that device.
float *scratch_on_current_device() {
  int dev = 0;
  MDP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) raise(MDP_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void *p = nullptr;
    MDP_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) raise(MDP_EHIP, "no device address for the scratch array");
    g_scratch[dev] = p;
  }
  return static_cast<float *>(g_scratch[dev]);
}

int64_t batch_max_unknowns() {
  const char *e = std::getenv("MDP_BATCH_MAX_UNKNOWNS");
  const long long v = e ? std::atoll(e) : 0;
  return v > 0 ? v : (int64_t{48} << 20);
}
}  // namespace

void set_last_error(const std::string &msg) { g_last_error = msg; }

AllocHook current_alloc_hook() {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  return g_hook;
}

void set_alloc_hook(const AllocHook &h) {
  std::lock_guard<std::mutex> lk(g_hook_mu);
  g_hook = h;
}

void *dev_alloc(size_t bytes, const AllocHook &h) {
  if (h.alloc) return h.alloc(bytes, h.ctx);
  void *p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return p;
}

void dev_free(void *p, const AllocHook &h) {
  if (h.free_)
    h.free_(p, h.ctx);
  else
    (void)hipFree(p);
}

int check_options(const mdp_options &o) {
  auto bad = [](const char *m) {
    set_last_error(m);
    return MDP_EINVAL;
  };
  if (o.precision != MDP_FP64 && o.precision != MDP_MIXED) return bad("precision must be MDP_FP64 or MDP_MIXED");
  if (o.vcycles < 1) return bad("vcycles must be >= 1");
  if (o.pre_sweeps < 1 || o.pre_sweeps > kMaxSweeps || o.post_sweeps < 1 || o.post_sweeps > kMaxSweeps)
    return bad("pre_sweeps and post_sweeps must be in [1, 8]");
  if (!(o.strength_theta >= 0.0)) return bad("strength_theta must be >= 0");
  if (o.max_coarse < 1 || o.max_dense < 0 || o.max_levels < 1) return bad("bad coarsening limits");
  if (o.restart < 1 || o.restart > kMaxCols) return bad("restart must be in [1, 64]");
  if (o.max_iter < 0) return bad("max_iter must be >= 0");
  if (!(o.rtol > 0.0)) return bad("rtol must be > 0");
  if (o.flags & ~(MDP_USE_X0 | MDP_HOST_ONLY | MDP_NO_AUTOTUNE | MDP_GRAPHS | MDP_FALLBACK_FP64 | MDP_HOST_PRODUCTS))
    return bad("unknown bits in flags");
  if (o.block_form != MDP_BLOCK_LOWER && o.block_form != MDP_BLOCK_DIAG && o.block_form != MDP_BLOCK_UPPER)
    return bad("block_form must be MDP_BLOCK_LOWER, MDP_BLOCK_DIAG or MDP_BLOCK_UPPER");
  if (o.smoother != MDP_SMOOTH_L1JACOBI && o.smoother != MDP_SMOOTH_GS)
    return bad("smoother must be MDP_SMOOTH_L1JACOBI or MDP_SMOOTH_GS");
  return MDP_OK;
}

namespace {

// Four-column plans of all handles together hold at most multi_rhs_cap()
// device bytes: MDP_MULTI_RHS_BYTES when set, else a quarter of the device's
// memory.  A handle whose plan does not fit solves its columns one at a time.
std::mutex g_mrhs_mu;
int64_t g_mrhs_held = 0;  // under g_mrhs_mu

int64_t multi_rhs_cap() {
  if (const char *e = std::getenv("MDP_MULTI_RHS_BYTES")) return std::max<int64_t>(0, std::atoll(e));
  static const int64_t quarter = [] {
    size_t fr = 0, tot = 0;
    if (hipMemGetInfo(&fr, &tot) != hipSuccess) {
      (void)hipGetLastError();
      return int64_t{0};
    }
    return static_cast<int64_t>(tot / 4);
  }();
  return quarter;
}

// One four-column Krylov workspace per device, shared by every handle's
// plan there: a plan keeps only its matrices.  The workspace grows to the
// largest plan's sizes; four-column solves on a device take turns on it.
struct SharedRhs4 {
  std::mutex use;     // held through a four-column solve and while the workspace changes
  Workspace ws;
  int64_t bytes = 0;  // device bytes of ws (counted in g_mrhs_held)
  int plans = 0;      // plans on this device (under g_mrhs_mu)
};
// never destroyed: the arrays stay until the process ends, as the runtime
// may be gone by the time static destructors run
SharedRhs4 &rhs4_of(int dev) {
  static SharedRhs4 *const all = new SharedRhs4[kMaxDevices];
  return all[dev];
}

size_t rhs4_tsz(const mdp_options &o) { return o.precision == MDP_MIXED ? sizeof(float) : sizeof(double); }

// Build h's four-column plan if the budget has room (see mdp_solve).
void build_multi_rhs(mdp_handle *h, hipStream_t s) {
  std::lock_guard<std::mutex> lk(g_mrhs_mu);
  const int64_t cap = multi_rhs_cap();
  if (g_mrhs_held >= cap || g_mrhs_held + h->rhs4_need > cap) return;
  int dev = 0;
  MDP_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) raise(MDP_EINVAL, "device index out of range");
  SharedRhs4 &sh = rhs4_of(dev);
  const int64_t before = t_dev_net_bytes;
  std::unique_ptr<Batch> bt;
  try {
    bt = std::make_unique<Batch>();
    bt->build(std::vector<const Solver *>(kMultiRhs, &h->s), s, false);
  } catch (const Error &e) {
    if (e.code != MDP_ENOMEM) throw;
    (void)hipGetLastError();  // clear the failed allocation's error state
    h->rhs4_failed = true;
    return;
  }
  const int64_t bytes = std::max<int64_t>(0, t_dev_net_bytes - before);
  // the shared workspace this plan needs, grown from what the device holds
  const int m = bt->opt.restart;
  const size_t tsz = rhs4_tsz(bt->opt);
  std::lock_guard<std::mutex> use(sh.use);
  const bool grow = !sh.ws.fits(bt->n, m, bt->npairs, bt->layout.ntiles, tsz);
  int64_t n_ws = bt->n;
  int np_ws = bt->npairs, nt_ws = bt->layout.ntiles;
  size_t tsz_ws = tsz;
  if (grow && sh.ws.allocated() && sh.ws.m == m) {
    n_ws = std::max<int64_t>(n_ws, sh.ws.ld);
    np_ws = std::max(np_ws, sh.ws.npairs);
    nt_ws = std::max(nt_ws, sh.ws.ntiles);
    tsz_ws = std::max(tsz_ws, sh.ws.tsz);
  }
  const int64_t ws_bytes =
      grow ? static_cast<int64_t>(Workspace::bytes_for(n_ws, m, np_ws, nt_ws, tsz_ws, true)) : sh.bytes;
  if (g_mrhs_held + bytes + (ws_bytes - sh.bytes) > cap) {
    h->rhs4_need = bytes + (ws_bytes - sh.bytes);
    return;
  }
  if (grow) {
    try {
      MDP_HIP(hipDeviceSynchronize());  // no plan's work may still use the old arrays
      sh.ws.release();
      sh.ws.alloc(n_ws, m, np_ws, nt_ws, tsz_ws, s);
      sh.ws.bp.alloc(static_cast<size_t>(sh.ws.ld) * sizeof(double));
      sh.ws.xp.alloc(static_cast<size_t>(sh.ws.ld) * sizeof(double));
    } catch (const Error &e) {
      sh.ws.release();
      g_mrhs_held -= sh.bytes;
      sh.bytes = 0;
      if (e.code != MDP_ENOMEM) throw;
      (void)hipGetLastError();
      h->rhs4_failed = true;
      return;
    }
    g_mrhs_held += ws_bytes - sh.bytes;
    sh.bytes = ws_bytes;
  }
  bt->wsp = &sh.ws;
  h->rhs4 = std::move(bt);
  h->rhs4_dev = dev;
  ++sh.plans;
  g_mrhs_held += bytes;
  h->rhs4_bytes = bytes;
}

}  // namespace

int solve_columns(mdp_handle *h, const std::vector<PairIO> &cols, hipStream_t s, mdp_stats *st, bool group,
                  int64_t *grouped) {
  const int32_t nrhs = static_cast<int32_t>(cols.size());
  int worst = MDP_OK;
  int32_t k = 0;
  auto fail_rest = [&](int32_t from, int rc) {
    for (int32_t r = from; r < nrhs; ++r) st[r].status = rc;
    return rc;
  };
  // Four columns at a time run as one batch of the same system, whose
  // sparse products read each matrix once for all four (the plan is built on
  // first use and kept with the handle); without room in the plans' budget,
  // or without device memory for it, the columns are solved one by one.
  if (group && nrhs >= kMultiRhs && !h->rhs4 && !h->rhs4_failed) build_multi_rhs(h, s);
  if (group && h->rhs4 && nrhs >= kMultiRhs) {
    std::lock_guard<std::mutex> use(rhs4_of(h->rhs4_dev).use);
    for (; k + kMultiRhs <= nrhs; k += kMultiRhs) {
      const std::vector<PairIO> io(cols.begin() + k, cols.begin() + k + kMultiRhs);
      int rc = h->rhs4->solve(io, s, st + k);
      if (grouped) *grouped += kMultiRhs;
      if ((h->s.opt.flags & MDP_FALLBACK_FP64) && h->s.opt.precision == MDP_MIXED) {
        // MDP_FALLBACK_FP64: columns of the group that produced a NaN/Inf or
        // stagnated are solved again, one by one, in FP64
        rc = MDP_OK;
        for (int r = 0; r < kMultiRhs; ++r) {
          mdp_stats &c = st[k + r];
          if (c.status == MDP_ENAN || c.status == MDP_STAGNATED) {
            mdp_stats again{};
            h->s.solve(cols[k + r].b, cols[k + r].x, s, &again, true);
            again.iters += c.iters;
            again.restarts += c.restarts + 1;
            c = again;
          }
          if (c.status < 0) {
            if (rc >= 0 || c.status < rc) rc = c.status;
          } else if (rc >= 0 && c.status > rc) {
            rc = c.status;
          }
        }
      }
      if (rc < 0) return fail_rest(k + kMultiRhs, rc);
      if (rc > worst) worst = rc;
    }
  }
  for (; k < nrhs; ++k) {
    const int rc = h->s.solve(cols[k].b, cols[k].x, s, st + k);
    if (rc < 0) return fail_rest(k + 1, rc);
    if (rc > worst) worst = rc;
  }
  return worst;
}

namespace {

// h's plan is going: its bytes leave the budget, and the device's shared
// workspace goes with the last plan there.
void drop_multi_rhs(mdp_handle *h) {
  if (!h->rhs4) return;
  std::lock_guard<std::mutex> lk(g_mrhs_mu);
  SharedRhs4 &sh = rhs4_of(h->rhs4_dev);
  g_mrhs_held -= h->rhs4_bytes;
  h->rhs4_bytes = 0;
  h->rhs4.reset();
  if (--sh.plans == 0) {
    std::lock_guard<std::mutex> use(sh.use);
    (void)hipDeviceSynchronize();
    sh.ws.release();
    g_mrhs_held -= sh.bytes;
    sh.bytes = 0;
  }
}

}  // namespace

}  // namespace mdp

using namespace mdp;

#define API_BEGIN try {
#define API_END                                                   \
  }                                                               \
  catch (const mdp::Error &e) {                                   \
    set_last_error(e.msg);                                        \
    return e.code;                                                \
  }                                                               \
  catch (const mdp::SetupError &e) {                              \
    set_last_error(e.msg);                                        \
    return e.code;                                                \
  }                                                               \
  catch (const std::bad_alloc &) {                                \
    set_last_error("host allocation failed");                     \
    return MDP_ENOMEM;                                            \
  }                                                               \
  catch (const std::exception &e) {                               \
    set_last_error(e.what());                                     \
    return MDP_EINVAL;                                            \
  }

extern "C" {

int mdp_options_default(mdp_options *o) {
  if (!o) {
    set_last_error("NULL options");
    return MDP_EINVAL;
  }
  o->precision = MDP_FP64;
  o->vcycles = 1;
  o->pre_sweeps = 1;
  o->post_sweeps = 1;
  o->strength_theta = 0.02;
  o->max_coarse = 400;
  o->max_dense = 2000;
  o->max_levels = 10;
  o->restart = 64;
  o->max_iter = 1000;
  o->rtol = 1e-8;
  o->flags = 0;
  o->block_form = MDP_BLOCK_LOWER;
  o->smoother = MDP_SMOOTH_L1JACOBI;
  return MDP_OK;
}

int mdp_setup(const mdp_csr *A, const int32_t *part, const mdp_options *opt, void *hip_stream, mdp_handle **out) {
  return mdp_setup_labeled(A, part, nullptr, opt, hip_stream, out);
}

int mdp_setup_labeled(const mdp_csr *A, const int32_t *part, const int32_t *label, const mdp_options *opt,
                      void *hip_stream, mdp_handle **out) {
  API_BEGIN
  if (!out) {
    set_last_error("NULL output handle");
    return MDP_EINVAL;
  }
  *out = nullptr;
  mdp_options o;
  if (opt)
    o = *opt;
  else
    mdp_options_default(&o);
  const int rc = check_options(o);
  if (rc != MDP_OK) return rc;
  const auto t0 = std::chrono::steady_clock::now();
  auto h = std::make_unique<mdp_handle>();
  h->s.opt = o;
  {
    const Range r("mdp_setup host");
    const DeviceProducts dp(!(o.flags & (MDP_HOST_ONLY | MDP_HOST_PRODUCTS)), hip_stream);
    build_host_system(A, part, o, h->s.host, label);
  }
  h->s.n = h->s.host.n;
  h->s.n_o = h->s.host.n_o;
  h->s.n_g = h->s.host.n_g;
  if (!(o.flags & MDP_HOST_ONLY)) {
    const Range r("mdp_setup upload");
    h->s.upload(static_cast<hipStream_t>(hip_stream));
  }
  h->s.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return MDP_OK;
  API_END
}

int mdp_setup_like(const mdp_handle *src, const mdp_options *opt, void *hip_stream, mdp_handle **out) {
  API_BEGIN
  if (!src || !opt || !out) {
    set_last_error("NULL argument");
    return MDP_EINVAL;
  }
  *out = nullptr;
  const mdp_options &o = *opt;
  const int rc = check_options(o);
  if (rc != MDP_OK) return rc;
  const mdp_options &so = src->s.opt;
  if (o.strength_theta != so.strength_theta || o.max_coarse != so.max_coarse || o.max_dense != so.max_dense ||
      o.max_levels != so.max_levels) {
    set_last_error("AMG options differ from the source handle");
    return MDP_EINVAL;
  }
  const auto t0 = std::chrono::steady_clock::now();
  auto h = std::make_unique<mdp_handle>();
  h->s.opt = o;
  h->s.host = src->s.host;
  h->s.n = h->s.host.n;
  h->s.n_o = h->s.host.n_o;
  h->s.n_g = h->s.host.n_g;
  if (!(o.flags & MDP_HOST_ONLY)) {
    const Range r("mdp_setup upload");
    h->s.upload(static_cast<hipStream_t>(hip_stream));
  }
  h->s.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return MDP_OK;
  API_END
}

int mdp_save(const mdp_handle *h, const char *path) {
  API_BEGIN
  if (!h || !path) {
    set_last_error("NULL argument");
    return MDP_EINVAL;
  }
  save_host_system(h->s.host, h->s.opt, path);
  return MDP_OK;
  API_END
}

int mdp_load(const char *path, const mdp_options *opt, void *hip_stream, mdp_handle **out) {
  API_BEGIN
  if (!path || !out) {
    set_last_error("NULL argument");
    return MDP_EINVAL;
  }
  *out = nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  auto h = std::make_unique<mdp_handle>();
  mdp_options saved;
  mdp_options_default(&saved);
  load_host_system(path, h->s.host, saved);
  mdp_options o = saved;
  if (opt) {
    o = *opt;
    if (o.strength_theta != saved.strength_theta || o.max_coarse != saved.max_coarse ||
        o.max_dense != saved.max_dense || o.max_levels != saved.max_levels) {
      set_last_error("AMG options differ from the ones the hierarchy file was built with");
      return MDP_EINVAL;
    }
  }
  const int rc = check_options(o);
  if (rc != MDP_OK) return rc;
  h->s.opt = o;
  h->s.n = h->s.host.n;
  h->s.n_o = h->s.host.n_o;
  h->s.n_g = h->s.host.n_g;
  if (!(o.flags & MDP_HOST_ONLY)) {
    const Range r("mdp_setup upload");
    h->s.upload(static_cast<hipStream_t>(hip_stream));
  }
  h->s.setup_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  *out = h.release();
  return MDP_OK;
  API_END
}

int mdp_destroy(mdp_handle *h) {
  API_BEGIN
  if (h) {
    std::lock_guard<std::mutex> lk(g_batch_mu);
    if (g_batch && std::find(g_batch->handles.begin(), g_batch->handles.end(), h) != g_batch->handles.end())
      g_batch.reset();
  }
  if (h) drop_multi_rhs(h);
  delete h;
  return MDP_OK;
  API_END
}

int mdp_residual_history(const mdp_handle *h, double *out, int32_t cap, int32_t *count) {
  API_BEGIN
  if (!h || cap < 0 || (cap > 0 && !out)) {
    set_last_error("bad history arguments");
    return MDP_EINVAL;
  }
  const std::vector<double> &hist = h->s.ws.history;
  if (count) *count = static_cast<int32_t>(hist.size());
  const size_t n = std::min(hist.size(), static_cast<size_t>(cap));
  std::copy(hist.begin(), hist.begin() + static_cast<std::ptrdiff_t>(n), out);
  return MDP_OK;
  API_END
}

int mdp_multi_rhs_memory(const mdp_handle *h, int64_t *plan_bytes, int64_t *shared_bytes, int64_t *held,
                         int64_t *budget) {
  API_BEGIN
  if (!h) {
    set_last_error("null handle");
    return MDP_EINVAL;
  }
  std::lock_guard<std::mutex> lk(g_mrhs_mu);
  if (plan_bytes) *plan_bytes = h->rhs4 ? h->rhs4_bytes : 0;
  if (shared_bytes) *shared_bytes = h->rhs4 ? rhs4_of(h->rhs4_dev).bytes : 0;
  if (held) *held = g_mrhs_held;
  if (budget) *budget = multi_rhs_cap();
  return MDP_OK;
  API_END
}

int mdp_solve(mdp_handle *h, const double *b, double *x, int32_t nrhs, int64_t ld, void *hip_stream,
              mdp_stats *stats) {
  API_BEGIN
  if (!h || !b || !x || nrhs < 0 || (nrhs > 1 && ld < h->s.n)) {
    set_last_error("bad solve arguments");
    return MDP_EINVAL;
  }
  if (!h->s.on_device) {
    set_last_error("handle was set up host-only");
    return MDP_EINVAL;
  }
  std::vector<PairIO> cols;
  for (int32_t k = 0; k < nrhs; ++k) cols.push_back(PairIO{b + k * ld, x + k * ld});
  std::vector<mdp_stats> st(static_cast<size_t>(nrhs));
  const int rc = solve_columns(h, cols, static_cast<hipStream_t>(hip_stream), st.data(), true);
  if (stats)
    for (int32_t k = 0; k < nrhs; ++k) stats[k] = st[k];
  return rc;
  API_END
}

int mdp_solve_batch(mdp_handle *const *hs, int32_t nsys, const double *const *b, double *const *x,
                    const int32_t *nrhs, void *hip_stream, mdp_stats *stats) {
  API_BEGIN
  if (!hs || !b || !x || !nrhs || nsys < 0) {
    set_last_error("bad batch arguments");
    return MDP_EINVAL;
  }
  std::vector<const Solver *> pairs;
  std::vector<mdp_handle *> pair_h;  // the handle of every pair (for the FP64 fallback)
  std::vector<PairIO> io;
  for (int32_t i = 0; i < nsys; ++i) {
    if (!hs[i] || nrhs[i] < 0 || (nrhs[i] > 0 && (!b[i] || !x[i]))) {  // no vectors needed for nrhs 0
      set_last_error("bad batch entry " + std::to_string(i));
      return MDP_EINVAL;
    }
    const Solver &s0 = hs[0]->s, &si = hs[i]->s;
    if (!si.on_device) {
      set_last_error("handle " + std::to_string(i) + " was set up host-only");
      return MDP_EINVAL;
    }
    if (si.opt.precision != s0.opt.precision || si.opt.vcycles != s0.opt.vcycles ||
        si.opt.pre_sweeps != s0.opt.pre_sweeps || si.opt.post_sweeps != s0.opt.post_sweeps ||
        si.opt.smoother != s0.opt.smoother ||
        si.opt.restart != s0.opt.restart || si.opt.max_iter != s0.opt.max_iter || si.opt.rtol != s0.opt.rtol ||
        si.opt.block_form != s0.opt.block_form ||
        (si.opt.flags & (MDP_USE_X0 | MDP_GRAPHS)) != (s0.opt.flags & (MDP_USE_X0 | MDP_GRAPHS))) {
      set_last_error("all handles of a batch need the same solve options");
      return MDP_EINVAL;
    }
    for (int32_t k = 0; k < nrhs[i]; ++k) {
      pairs.push_back(&si);
      pair_h.push_back(hs[i]);
      io.push_back(PairIO{b[i] + static_cast<int64_t>(k) * si.n, x[i] + static_cast<int64_t>(k) * si.n});
    }
  }
  if (pairs.empty()) return MDP_OK;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  std::lock_guard<std::mutex> lk(g_batch_mu);
  const std::vector<const mdp_handle *> key_h(hs, hs + nsys);
  const std::vector<int32_t> key_r(nrhs, nrhs + nsys);
  const int64_t cap = batch_max_unknowns();
  if (!g_batch || g_batch->handles != key_h || g_batch->nrhs != key_r || g_batch->cap != cap) {
    g_batch.reset();
    auto bc = std::make_unique<BatchCache>();
    bc->handles = key_h;
    bc->nrhs = key_r;
    bc->cap = cap;
    // Chunks of at most `cap` unknowns (or one pair), cut between systems
    // where possible, so that a system's right-hand sides stay in one chunk
    // and share its preconditioner's matrix reads; a system whose right-hand
    // sides exceed `cap` together is split between them.
    std::vector<std::pair<size_t, size_t>> cuts;
    size_t p0 = 0, pi = 0;
    int64_t tot = 0;
    auto cut = [&] {
      if (pi > p0) cuts.emplace_back(p0, pi);
      p0 = pi;
      tot = 0;
    };
    for (int32_t i = 0; i < nsys; ++i) {
      if (nrhs[i] == 0) continue;
      const int64_t ni = hs[i]->s.n, group = ni * nrhs[i];
      if (tot + group > cap) cut();
      if (group <= cap) {
        tot += group;
        pi += static_cast<size_t>(nrhs[i]);
        continue;
      }
      for (int32_t k = 0; k < nrhs[i]; ++k) {
        if (tot + ni > cap) cut();
        tot += ni;
        ++pi;
      }
    }
    cut();
    for (const auto &c : cuts) {
      auto bt = std::make_unique<Batch>();
      bt->build(std::vector<const Solver *>(pairs.begin() + c.first, pairs.begin() + c.second), s, false);
      bc->first_pair.push_back(static_cast<int>(c.first));
      bc->chunks.push_back(std::move(bt));
    }
    int64_t nmax = 0;
    int pmax = 0, tmax = 0;
    for (const auto &bt : bc->chunks) {
      nmax = std::max<int64_t>(nmax, bt->n);
      pmax = std::max(pmax, bt->npairs);
      tmax = std::max(tmax, bt->layout.ntiles);
    }
    const mdp_options &o = bc->chunks[0]->opt;
    bc->shared.alloc(nmax, o.restart, pmax, tmax, o.precision == MDP_MIXED ? sizeof(float) : sizeof(double), s);
    bc->shared.bp.alloc(static_cast<size_t>(bc->shared.ld) * sizeof(double));
    bc->shared.xp.alloc(static_cast<size_t>(bc->shared.ld) * sizeof(double));
    for (auto &bt : bc->chunks) bt->wsp = &bc->shared;
    g_batch = std::move(bc);
  }
  int worst = MDP_OK;
  auto fold = [&](int rc) {
    if (rc < 0) {
      if (worst >= 0 || rc < worst) worst = rc;
    } else if (worst >= 0 && rc > worst) {
      worst = rc;
    }
  };
  std::vector<mdp_stats> st(pairs.size());
  for (size_t c = 0; c < g_batch->chunks.size(); ++c) {
    Batch &bt = *g_batch->chunks[c];
    const int p0 = g_batch->first_pair[c];
    const std::vector<PairIO> sub(io.begin() + p0, io.begin() + p0 + bt.npairs);
    const int rc = bt.solve(sub, s, st.data() + p0);
    if (rc >= 0 || rc == MDP_ENAN) {
      // MDP_FALLBACK_FP64 (mixed): pairs that produced a NaN/Inf or
      // stagnated are solved again, one by one, with their handle's FP64
      // preconditioner
      for (int q = p0; q < p0 + bt.npairs; ++q) {
        mdp_stats &cs = st[q];
        Solver &sv = pair_h[q]->s;
        if ((cs.status == MDP_ENAN || cs.status == MDP_STAGNATED) && sv.opt.precision == MDP_MIXED &&
            (sv.opt.flags & MDP_FALLBACK_FP64)) {
          mdp_stats again{};
          sv.solve(io[q].b, io[q].x, s, &again, true);
          again.iters += cs.iters;
          again.restarts += cs.restarts + 1;
          cs = again;
        }
        fold(cs.status);
      }
    } else {
      fold(rc);
    }
  }
  if (stats)
    for (size_t q = 0; q < st.size(); ++q) stats[q] = st[q];
  return worst;
  API_END
}

int mdp_apply(mdp_handle *h, int32_t op, const double *x, double *y, void *hip_stream) {
  API_BEGIN
  if (!h || !x || !y) {
    set_last_error("bad apply arguments");
    return MDP_EINVAL;
  }
  if (!h->s.on_device) {
    set_last_error("handle was set up host-only");
    return MDP_EINVAL;
  }
  h->s.apply(op, x, y, static_cast<hipStream_t>(hip_stream));
  return MDP_OK;
  API_END
}

int mdp_apply_noalloc(mdp_handle *h, int32_t op, const double *x, double *y, void *hip_stream) {
  API_BEGIN
  if (!h || !x || !y) {
    set_last_error("bad apply arguments");
    return MDP_EINVAL;
  }
  if (op != MDP_OP_A && op != MDP_OP_ML && op != MDP_OP_QOO && op != MDP_OP_QGG) {
    set_last_error("unknown operator");
    return MDP_EINVAL;
  }
  const int64_t len = op == MDP_OP_QOO ? h->s.n_o : (op == MDP_OP_QGG ? h->s.n_g : h->s.n);
  const bool staged = h->s.opt.precision == MDP_MIXED && op != MDP_OP_A;
  if (staged && 2 * len * static_cast<int64_t>(sizeof(float)) > static_cast<int64_t>(kScratchBytes)) {
    set_last_error("operator of " + std::to_string(len) + " unknowns exceeds the no-allocation limit of " +
                   std::to_string(kScratchBytes / (2 * sizeof(float))) + " in mixed precision");
    return MDP_EINVAL;
  }
  if (!h->s.on_device) {
    set_last_error("handle was set up host-only");
    return MDP_EINVAL;
  }
  if (ktimer_any_on()) {
    set_last_error("kernel timers are running (they create events); stop them first");
    return MDP_EINVAL;
  }
  float *in = scratch_on_current_device();
  h->s.enqueue_apply(op, x, y, static_cast<hipStream_t>(hip_stream), in, in + len);
  return MDP_OK;
  API_END
}

int mdp_info(const mdp_handle *h, int32_t *n, int32_t *no, int32_t *ng, int32_t *lo, int32_t *lg) {
  if (!h) {
    set_last_error("NULL handle");
    return MDP_EINVAL;
  }
  if (n) *n = h->s.host.n;
  if (no) *no = h->s.host.n_o;
  if (ng) *ng = h->s.host.n_g;
  if (lo) *lo = static_cast<int32_t>(h->s.host.Ho.lv.size());
  if (lg) *lg = static_cast<int32_t>(h->s.host.Hg.lv.size());
  return MDP_OK;
}

static const HCsr *pick(const mdp_handle *h, int32_t block, int32_t level, int32_t mat) {
  if (!h) return nullptr;
  const HHier &H = block == MDP_BLOCK_OMEGA ? h->s.host.Ho : h->s.host.Hg;
  if (block != MDP_BLOCK_OMEGA && block != MDP_BLOCK_GAMMA) return nullptr;
  if (level < 0 || level >= static_cast<int32_t>(H.lv.size())) return nullptr;
  const bool last = level + 1 == static_cast<int32_t>(H.lv.size());
  if (mat == MDP_MAT_A) return &H.lv[level].A;
  if (last) return nullptr;
  if (mat == MDP_MAT_P) return &H.lv[level].P;
  if (mat == MDP_MAT_R) return &H.lv[level].R;
  return nullptr;
}

int mdp_level_shape(const mdp_handle *h, int32_t block, int32_t level, int32_t mat, int32_t *rows, int32_t *cols,
                    int64_t *nnz) {
  const HCsr *m = pick(h, block, level, mat);
  if (!m) {
    set_last_error("no such hierarchy matrix");
    return MDP_EINVAL;
  }
  if (rows) *rows = m->nr;
  if (cols) *cols = m->nc;
  if (nnz) *nnz = m->nnz();
  return MDP_OK;
}

int mdp_level_export(const mdp_handle *h, int32_t block, int32_t level, int32_t mat, int32_t *row_ptr,
                     int32_t *col, double *val) {
  const HCsr *m = pick(h, block, level, mat);
  if (!m || !row_ptr || (m->nnz() > 0 && (!col || !val))) {
    set_last_error("no such hierarchy matrix or NULL buffer");
    return MDP_EINVAL;
  }
  std::copy(m->ptr.begin(), m->ptr.end(), row_ptr);
  std::copy(m->col.begin(), m->col.end(), col);
  std::copy(m->val.begin(), m->val.end(), val);
  return MDP_OK;
}

int mdp_level_aggregates(const mdp_handle *h, int32_t block, int32_t level, int32_t *agg) {
  if (!pick(h, block, level, MDP_MAT_P) || !agg) {
    set_last_error("level has no aggregates");
    return MDP_EINVAL;
  }
  const HHier &H = block == MDP_BLOCK_OMEGA ? h->s.host.Ho : h->s.host.Hg;
  std::copy(H.lv[level].agg.begin(), H.lv[level].agg.end(), agg);
  return MDP_OK;
}

int mdp_tune_file(const char *path) {
  API_BEGIN
  set_tune_file(path);
  return MDP_OK;
  API_END
}

int mdp_set_allocator(void *(*alloc)(size_t, void *), void (*free_)(void *, void *), void *ctx) {
  if ((alloc == nullptr) != (free_ == nullptr)) {
    set_last_error("alloc and free must both be set or both be NULL");
    return MDP_EINVAL;
  }
  AllocHook hk;
  hk.alloc = alloc;
  hk.free_ = free_;
  hk.ctx = ctx;
  set_alloc_hook(hk);
  return MDP_OK;
}

const char *mdp_last_error(void) { return g_last_error.c_str(); }

const char *mdp_version(void) { return "mdp 0.1 (gfx950)"; }

}  // extern "C"
