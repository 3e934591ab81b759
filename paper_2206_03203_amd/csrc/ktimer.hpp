// Kernel-class timers: HIP events recorded around each launch of a class on
// the stream it is launched on, with the algorithmic bytes of that launch
// (every matrix value and index once, every vector once).  Off by default.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace mdp {

enum KClass : int {
  kKcOuterSpmv = 0,    // w = A z_j, FP64 system matrix
  kKcFineSmooth = 1,   // finest S~ level: sweeps after the first (post-smoothing, extra pre-smoothing)
  kKcVcycleOther = 2,  // other V-cycle kernels (restriction, prolongation, coarser levels, A_GG, A_GO)
  kKcArnoldiDot = 3,   // fused reduction pass of the Arnoldi step
  kKcArnoldiAxpy = 4,  // update pass of the Arnoldi step
  kKcOther = 5,        // casts, small reductions, Givens, solution update, residual
  kKcFineResid = 6,    // finest S~ level: residual after the first sweep (fused: its restriction)
  kKcCount = 7
};

bool ktimer_on(int kind);
bool ktimer_any_on();

// Algorithmic-byte counters, saved before a batch of launches and restored
// when those launches turn out to be retired no-ops (gated after
// convergence): their time still counts, their bytes do not.
struct KtBytes {
  double b[kKcCount];
};
KtBytes ktimer_bytes();
void ktimer_restore_bytes(const KtBytes &s);
// Correct the bytes of class `kind` once the work its launches skipped is known.
void ktimer_add_bytes(int kind, double delta);
// Returns the event pair to record around the next launch of `kind`.
void ktimer_pair(int kind, double bytes, hipEvent_t *start, hipEvent_t *stop);

// Run `launch` bracketed by timing events when the class is enabled.
template <typename F>
inline void timed_launch(int kind, hipStream_t s, double bytes, F &&launch) {
  if (!ktimer_on(kind)) {
    launch();
    return;
  }
  hipEvent_t a, b;
  ktimer_pair(kind, bytes, &a, &b);
  (void)hipEventRecord(a, s);
  launch();
  (void)hipEventRecord(b, s);
}

}  // namespace mdp
