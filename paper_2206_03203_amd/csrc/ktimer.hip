// Kernel-class timer registry (see ktimer.hpp) and its C entry points.
#include <mutex>
#include <vector>

#include "ktimer.hpp"
#include "mdp.h"
#include "runtime.hpp"

namespace mdp {

namespace {
struct Registry {
  std::mutex mu;
  bool on[kKcCount] = {};
  std::vector<hipEvent_t> ev[kKcCount];  // start/stop pairs, grown on demand
  size_t used[kKcCount] = {};
  double bytes[kKcCount] = {};
};
Registry &reg() {
  static Registry r;
  return r;
}
}  // namespace

bool ktimer_on(int kind) { return reg().on[kind]; }

bool ktimer_any_on() {
  for (int k = 0; k < kKcCount; ++k)
    if (reg().on[k]) return true;
  return false;
}

KtBytes ktimer_bytes() {
  Registry &r = reg();
  std::lock_guard<std::mutex> lk(r.mu);
  KtBytes s;
  for (int k = 0; k < kKcCount; ++k) s.b[k] = r.bytes[k];
  return s;
}

void ktimer_restore_bytes(const KtBytes &s) {
  Registry &r = reg();
  std::lock_guard<std::mutex> lk(r.mu);
  for (int k = 0; k < kKcCount; ++k)
    if (r.on[k]) r.bytes[k] = s.b[k];
}

void ktimer_add_bytes(int kind, double delta) {
  Registry &r = reg();
  std::lock_guard<std::mutex> lk(r.mu);
  if (r.on[kind]) r.bytes[kind] += delta;
}

void ktimer_pair(int kind, double bytes, hipEvent_t *start, hipEvent_t *stop) {
  Registry &r = reg();
  std::lock_guard<std::mutex> lk(r.mu);
  auto &v = r.ev[kind];
  const size_t k = r.used[kind];
  while (v.size() < 2 * (k + 1)) {
    hipEvent_t e;
    MDP_HIP(hipEventCreate(&e));
    v.push_back(e);
  }
  *start = v[2 * k];
  *stop = v[2 * k + 1];
  r.used[kind] = k + 1;
  r.bytes[kind] += bytes;
}

}  // namespace mdp

using namespace mdp;

extern "C" {

int mdp_ktimer_begin(int32_t kind) {
  if (kind < 0 || kind >= kKcCount) {
    set_last_error("unknown kernel class");
    return MDP_EINVAL;
  }
  Registry &r = reg();
  std::lock_guard<std::mutex> lk(r.mu);
  r.on[kind] = true;
  r.used[kind] = 0;
  r.bytes[kind] = 0.0;
  return MDP_OK;
}

int mdp_ktimer_end(int32_t kind, double *total_ms, int64_t *launches, double *bytes) {
  if (kind < 0 || kind >= kKcCount) {
    set_last_error("unknown kernel class");
    return MDP_EINVAL;
  }
  Registry &r = reg();
  std::lock_guard<std::mutex> lk(r.mu);
  r.on[kind] = false;
  double ms = 0.0;
  for (size_t k = 0; k < r.used[kind]; ++k) {
    float t = 0.f;
    hipEvent_t a = r.ev[kind][2 * k], b = r.ev[kind][2 * k + 1];
    if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&t, a, b) != hipSuccess) {
      set_last_error("event timing failed");
      return MDP_EHIP;
    }
    ms += t;
  }
  if (total_ms) *total_ms = ms;
  if (launches) *launches = static_cast<int64_t>(r.used[kind]);
  if (bytes) *bytes = r.bytes[kind];
  return MDP_OK;
}

}  // extern "C"
