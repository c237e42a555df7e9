// Device building blocks of the Fourier kernels (internal).
#pragma once
#include "kernels.h"

namespace rbe {

// Phase of mode m at fractional coordinate s, in turns, reduced to
// [-1/2, 1/2]: t = m . s - rint(m . s) (FP64, the dot product with fused
// multiply-adds).
__device__ inline double turn_fraction(double mx, double my, double mz, double sx, double sy, double sz) {
  const double t = fma(mx, sx, fma(my, sy, mz * sz));
  return t - rint(t);
}

// The same phase as an FP32 argument of the hardware sin/cos, which take
// turns: any representative of m . s mod 1 serves, so the reduction is the
// fractional part in [0, 1) (one instruction), then rounded to FP32 (at most
// 2^-25 turns off).
__device__ inline float turn_f32(double mx, double my, double mz, double sx, double sy, double sz) {
  const double t = fma(mx, sx, fma(my, sy, mz * sz));
  return (float)__builtin_amdgcn_fract(t);
}

// sin and cos of 2 pi t for |t| <= 1/2 (FP64): u = 4t and f = u - rint(u)
// are exact, theta = f pi/2 lies in [-pi/4, pi/4], sin theta and cos theta
// come from their Taylor series to degrees 15 and 16 (truncation below
// 5e-17), and the result is rotated by the rint(u) quarter turns.
__device__ inline void sincos_turn_f64(double t, double *sn, double *cs) {
  const double u = 4.0 * t;
  const double q = rint(u);
  const double th = (u - q) * 1.5707963267948966;
  const double t2 = th * th;
  double ps = -7.647163731819816e-13;
  ps = fma(ps, t2, 1.6059043836821613e-10);
  ps = fma(ps, t2, -2.505210838544172e-08);
  ps = fma(ps, t2, 2.7557319223985893e-06);
  ps = fma(ps, t2, -0.0001984126984126984);
  ps = fma(ps, t2, 0.008333333333333333);
  ps = fma(ps, t2, -0.16666666666666666);
  ps = fma(ps * t2, th, th);
  double pc = 4.779477332387385e-14;
  pc = fma(pc, t2, -1.1470745597729725e-11);
  pc = fma(pc, t2, 2.08767569878681e-09);
  pc = fma(pc, t2, -2.755731922398589e-07);
  pc = fma(pc, t2, 2.48015873015873e-05);
  pc = fma(pc, t2, -0.001388888888888889);
  pc = fma(pc, t2, 0.041666666666666664);
  pc = fma(pc, t2, -0.5);
  pc = fma(pc, t2, 1.0);
  const int k = (int)q & 3;  // quarter turns, q in [-2, 2]
  const double a = (k & 1) ? pc : ps, b = (k & 1) ? ps : pc;
  *sn = (k & 2) ? -a : a;
  *cs = (k == 1 || k == 2) ? -b : b;
}

// sin and cos of 2 pi t for |t| <= 1/2 (FP64) from a table of the
// kTurnTable-th turns: j = rint(N t) and f = N t - j are exact (N a power of
// two), theta = 2 pi f / N lies in [-pi/N, pi/N], its sine and cosine come
// from Taylor polynomials of degrees 5 and 6 (truncation below 1e-17 for
// N = 256), and the angle-addition formulas combine them with the table's
// (sin, cos) of 2 pi j / N. tab is the table in LDS.
constexpr int kTurnTable = kTurnTableEntries;
__device__ inline void sincos_turn_tab_f64(double t, const double2 *tab, double *sn, double *cs) {
  const double u = t * (double)kTurnTable;
  const double j = rint(u);
  const double th = (u - j) * (6.283185307179586 / kTurnTable);
  const double t2 = th * th;
  const double s = fma(fma(t2, 1.0 / 120.0, -1.0 / 6.0) * t2, th, th);
  const double c = fma(fma(fma(t2, -1.0 / 720.0, 1.0 / 24.0), t2, -0.5), t2, 1.0);
  const double2 e = tab[(int)j & (kTurnTable - 1)];  // (sin, cos) of 2 pi j / N
  *sn = fma(e.x, c, e.y * s);
  *cs = fma(e.y, c, -(e.x * s));
}

// Kahan-compensated FP32 sum of products: sum += a b, with the product
// fused into the compensation step (one rounding instead of two).
__device__ inline void kahan_fma(float &sum, float &comp, float a, float b) {
#pragma clang fp contract(off)
  const float y = fmaf(a, b, -comp);
  const float t = sum + y;
  comp = (t - sum) - y;
  sum = t;
}

// FP32 copies of a mode's gather coefficients.
__device__ inline void gather_floats(GatherMode &gm) {
  gm.af = (float)gm.a;
  gm.bf = (float)gm.b;
  gm.mxf = (float)gm.mx;
  gm.myf = (float)gm.my;
  gm.mzf = (float)gm.mz;
  gm.pad = 0.f;
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
