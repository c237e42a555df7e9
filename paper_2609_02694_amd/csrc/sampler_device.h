// Mode draw of the importance sample (internal, host and device).
#pragma once
#include "rbe_internal.h"

namespace rbe {

// First index i of cdf[0..len) with u < cdf[i] (cdf nondecreasing, last = 1 > u).
__host__ __device__ inline int upper_index(const double *cdf, int len, double u) {
  int lo = 0, hi = len - 1;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (u < cdf[mid]) hi = mid;
    else lo = mid + 1;
  }
  return lo;
}

__host__ __device__ inline double mode_weight(const ModeTable &t, int P, int mx, int my, int mz) {
#pragma clang fp contract(off)
  const double kx = kTwoPi * (double)mx / t.L[0];
  const double ky = kTwoPi * (double)my / t.L[1];
  const double kz = kTwoPi * (double)mz / t.L[2];
  const double k2 = kx * kx + ky * ky + kz * kz;
  return (t.S / (double)P) * (4.0 * kPi / (t.V * k2));
}

constexpr int kMaxAttempts = 4096;

// Draw mode l; returns false if every attempt gave m = 0.
__host__ __device__ inline bool draw_mode(const ModeTable &t, const double *cdf, uint64_t eval_key, int l, int *mv) {
  const uint64_t kl = stream_out(eval_key, (uint64_t)l);
  for (int a = 0; a < kMaxAttempts; ++a) {
    for (int d = 0; d < 3; ++d) {
      const double u = unit53(stream_out(kl, (uint64_t)(3 * a + d)));
      mv[d] = upper_index(cdf + t.off[d], 2 * t.M[d] + 1, u) - t.M[d];
    }
    if (mv[0] != 0 || mv[1] != 0 || mv[2] != 0) return true;
  }
  return false;
}

}  // namespace rbe
