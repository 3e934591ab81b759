// Device runtime helpers: error propagation, the pluggable device allocator
// and owning device buffers.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "mdp.h"

namespace mdp {

struct Error {
  int code;
  std::string msg;
};

[[noreturn]] inline void raise(int code, const std::string &msg) { throw Error{code, msg}; }

#define MDP_HIP(expr)                                                                   \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      ::mdp::raise(e_ == hipErrorOutOfMemory ? MDP_ENOMEM : MDP_EHIP,                   \
                   std::string(#expr) + ": " + hipGetErrorString(e_));                  \
  } while (0)

void set_last_error(const std::string &msg);

// A named host-side range (setup, solve, restart cycle, preconditioner and
// Arnoldi enqueue) for tools that record ROCTx markers; next to nothing
// when none is attached.
struct Range {
  explicit Range(const char *name) { roctxRangePush(name); }
  ~Range() { roctxRangePop(); }
  Range(const Range &) = delete;
  Range &operator=(const Range &) = delete;
};

// Allocation goes through a process-wide hook (hipMalloc unless the caller
// installed its own allocator).  Each allocation remembers the hook that
// made it, so a later change of allocator frees old blocks correctly.
struct AllocHook {
  void *(*alloc)(size_t, void *) = nullptr;
  void (*free_)(void *, void *) = nullptr;
  void *ctx = nullptr;
};
AllocHook current_alloc_hook();
void set_alloc_hook(const AllocHook &h);
void *dev_alloc(size_t bytes, const AllocHook &h);
void dev_free(void *p, const AllocHook &h);

// Net device bytes this thread has allocated minus freed through DevMem: the
// difference across a build is what the built object keeps.
inline thread_local int64_t t_dev_net_bytes = 0;

// Owning, untyped device allocation.
class DevMem {
 public:
  DevMem() = default;
  explicit DevMem(size_t bytes) { alloc(bytes); }
  ~DevMem() { reset(); }
  DevMem(const DevMem &) = delete;
  DevMem &operator=(const DevMem &) = delete;
  DevMem(DevMem &&o) noexcept : p_(o.p_), n_(o.n_), hook_(o.hook_) {
    o.p_ = nullptr;
    o.n_ = 0;
  }
  DevMem &operator=(DevMem &&o) noexcept {
    if (this != &o) {
      reset();
      p_ = o.p_;
      n_ = o.n_;
      hook_ = o.hook_;
      o.p_ = nullptr;
      o.n_ = 0;
    }
    return *this;
  }
  void alloc(size_t bytes) {
    reset();
    if (bytes == 0) return;
    hook_ = current_alloc_hook();
    p_ = dev_alloc(bytes, hook_);
    if (!p_) raise(MDP_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
    n_ = bytes;
    t_dev_net_bytes += static_cast<int64_t>(bytes);
  }
  void reset() {
    if (p_) {
      dev_free(p_, hook_);
      t_dev_net_bytes -= static_cast<int64_t>(n_);
    }
    p_ = nullptr;
    n_ = 0;
  }
  template <typename T>
  T *as() const {
    return static_cast<T *>(p_);
  }
  void *get() const { return p_; }
  size_t bytes() const { return n_; }

 private:
  void *p_ = nullptr;
  size_t n_ = 0;
  AllocHook hook_;
};

template <typename T>
inline T *dptr(const DevMem &m) {
  return static_cast<T *>(m.get());
}

// Owning array of timing events.
class Events {
 public:
  explicit Events(size_t n) : ev_(n, nullptr) {
    try {
      for (auto &e : ev_) MDP_HIP(hipEventCreate(&e));
    } catch (...) {
      release();
      throw;
    }
  }
  ~Events() { release(); }
  Events(const Events &) = delete;
  Events &operator=(const Events &) = delete;
  hipEvent_t operator[](size_t i) const { return ev_[i]; }

 private:
  void release() {
    for (auto &e : ev_)
      if (e) (void)hipEventDestroy(e), e = nullptr;
  }
  std::vector<hipEvent_t> ev_;
};

// Round a vector length up so that consecutive columns start 256-byte aligned.
inline int64_t padded_ld(int64_t n) { return (n + 63) / 64 * 64; }

}  // namespace mdp
