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

__host__ __device__ inline double mode_k2(const ModeTable &t, int mx, int my, int mz) {
#pragma clang fp contract(off)
  const double kx = kTwoPi * (double)mx / t.L[0];
  const double ky = kTwoPi * (double)my / t.L[1];
  const double kz = kTwoPi * (double)mz / t.L[2];
  return kx * kx + ky * ky + kz * kz;
}

// Weight of a drawn mode: (S/P) 4 pi / (V k^2) for the Gaussian proposal;
// (S2/P) 4 pi / V for exp(-k^2/(4 alpha))/k^2, whose 1/k^2 cancels the
// one of the force.
__host__ __device__ inline double mode_weight(const ModeTable &t, int P, int mx, int my, int mz) {
#pragma clang fp contract(off)
  if (t.kdist == RBE_KDIST_GAUSS_OVER_K2) return (t.S2 / (double)P) * (4.0 * kPi / t.V);
  return (t.S / (double)P) * (4.0 * kPi / (t.V * mode_k2(t, mx, my, mz)));
}

constexpr int kMaxAttempts = 4096;
constexpr int kMaxAttemptsOverK2 = 1 << 20;

// Draw mode l; returns false if every attempt failed. Gaussian proposal:
// attempt a takes outputs 3a..3a+2 (one per axis, inverse CDF) and is
// rejected if m = 0. exp(-k^2/(4 alpha))/k^2: attempt a takes outputs
// 4a..4a+2 the same way and output 4a+3 = u, and is accepted if m != 0 and
// u k^2 < k_min^2 (probability k_min^2/k^2 <= 1, which turns the Gaussian
// proposal into the target exactly).
__host__ __device__ inline bool draw_mode(const ModeTable &t, const double *cdf, uint64_t eval_key, int l, int *mv) {
#pragma clang fp contract(off)
  const uint64_t kl = stream_out(eval_key, (uint64_t)l);
  const bool over_k2 = t.kdist == RBE_KDIST_GAUSS_OVER_K2;
  const int per = over_k2 ? 4 : 3;
  const int cap = over_k2 ? kMaxAttemptsOverK2 : kMaxAttempts;
  for (int a = 0; a < cap; ++a) {
    for (int d = 0; d < 3; ++d) {
      const double u = unit53(stream_out(kl, (uint64_t)per * (uint64_t)a + (uint64_t)d));
      mv[d] = upper_index(cdf + t.off[d], 2 * t.M[d] + 1, u) - t.M[d];
    }
    if (mv[0] == 0 && mv[1] == 0 && mv[2] == 0) continue;
    if (!over_k2) return true;
    const double u = unit53(stream_out(kl, (uint64_t)per * (uint64_t)a + 3u));
    if (u * mode_k2(t, mv[0], mv[1], mv[2]) < t.kmin2) return true;
  }
  return false;
}

}  // namespace rbe
