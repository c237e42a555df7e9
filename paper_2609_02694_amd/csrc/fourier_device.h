// Device building blocks of the Fourier kernels (internal).
#pragma once
#include "kernels.h"

namespace rbe {

// Phase of mode m at fractional coordinate s, in turns, reduced to
// [-1/2, 1/2]: t = m . s - rint(m . s) (FP64, no contraction).
__device__ inline double turn_fraction(double mx, double my, double mz, double sx, double sy, double sz) {
#pragma clang fp contract(off)
  const double t = mx * sx + my * sy + mz * sz;
  return t - rint(t);
}

// Kahan-compensated FP32 sum.
__device__ inline void kahan_add(float &sum, float &comp, float v) {
#pragma clang fp contract(off)
  const float y = v - comp;
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

}  // namespace rbe
