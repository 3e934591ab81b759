// Constants and device-visible structs shared by host and kernel code.
#pragma once

#include <cstdint>

namespace mdp {

constexpr int kThreads = 256;
constexpr int kXcds = 8;
constexpr int kRedBlocks = 1024;  // fixed number of partial sums per reduction
constexpr int kMaxCols = 64;      // Krylov basis columns handled by one Arnoldi pass

// Per-cycle FGMRES state in device memory.
struct GmresState {
  int done;      // set: later kernels of this cycle return at once
  int k;         // Arnoldi steps completed in this cycle
  int nan;       // a non-finite value appeared
  int breakdown; // h_{k+1,k} == 0
  double est;    // |g_k| (absolute residual estimate)
  double beta;   // residual norm at the cycle start
};

}  // namespace mdp
