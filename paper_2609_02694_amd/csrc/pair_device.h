// Device building blocks of the near-field kernels (internal): pair
// scalars of Eq. 8 in FP64 and FP32, compensated accumulation, and the
// stencil traversals of the cell list.
#pragma once
#include "kernels.h"

namespace rbe {

// Coefficients of the FP64 polynomials below, highest degree first.
#define RBE_ERFCX_COEFS \
    1.63618628481317543e-08, -4.60928758649811430e-08, -6.88442333452307132e-08, \
    4.40190654889049080e-07, -4.46917185831068957e-07, -1.14063358111397811e-06, \
    3.75537844601685302e-06, -1.41703053499259700e-06, -1.39602653735770222e-05, \
    2.75867068654632672e-05, 2.75241444094816018e-05, -1.74362281120596591e-04, \
    4.35557661104548185e-05, 9.81977137355043118e-04, -8.47143262890503600e-04, \
    -6.99746174546772310e-03, 3.73289240473987467e-03, 7.89785810158994406e-02, \
    2.41658194242463487e-01, 4.27185847413955655e-01, 2.55395676310504194e-01
#define RBE_EXP_COEFS \
    1.1470745597729725e-11, 1.6059043836821613e-10, 2.08767569878681e-09, 2.505210838544172e-08, \
    2.755731922398589e-07, 2.7557319223985893e-06, 2.48015873015873e-05, 0.0001984126984126984, \
    0.001388888888888889, 0.008333333333333333, 0.041666666666666664, 0.16666666666666666, 0.5, 1.0, \
    1.0
constexpr double kErfcxCoef[] = {RBE_ERFCX_COEFS};
constexpr double kExpCoef[] = {RBE_EXP_COEFS};
constexpr int kErfcxTerms = (int)(sizeof(kErfcxCoef) / sizeof(double));
constexpr int kExpTerms = (int)(sizeof(kExpCoef) / sizeof(double));
// The same coefficients in constant memory, for kernels that evaluate the
// pair scalar in a branch most trips of a neighbour walk skip: read there
// with scalar loads at an opaque offset, so the compiler cannot keep the
// whole table in vector registers for the walk (it did, costing a wave of
// occupancy).
static __constant__ double kErfcxTable[kErfcxTerms] = {RBE_ERFCX_COEFS};
static __constant__ double kExpTable[kExpTerms] = {RBE_EXP_COEFS};
__device__ inline int opaque_zero() {
  int z;
  asm volatile("s_mov_b32 %0, 0" : "=s"(z));
  return z;
}
// d = a b + c as one v_fma_f64 with c in vector (fma_vv) or scalar (fma_vs)
// registers; plain fma() here becomes v_fmac with the addend copied into the
// destination first, two or three instructions per polynomial step.
__device__ inline double fma_vv(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "v"(c));
  return d;
}
__device__ inline double fma_vs(double a, double b, double c) {
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
}
// Horner evaluation of a coefficient list at x (TABLE: from constant memory).
template <bool TABLE, int N>
__device__ inline double horner_f64(const double (&coef)[N], const double *table, double x) {
  if constexpr (TABLE) {
    const double *t = table + opaque_zero();
    double c[N];
#pragma unroll
    for (int k = 0; k < N; ++k) c[k] = t[k];  // issued together, merged into wide scalar loads
    double r = c[0];
#pragma unroll
    for (int k = 1; k < N; ++k) r = fma_vs(r, x, c[k]);
    return r;
  } else {
    double r = coef[0];
#pragma unroll
    for (int k = 1; k < N; ++k) r = fma_vv(r, x, coef[k]);
    return r;
  }
}

// FP64 erfc(x) = exp(-x^2) R(x) with R(x) = erfc(x) e^{x^2} a degree-20
// polynomial in s = 2/(1 + x/2) - 1 (fit over x in [0, 8] by fit_erfcx.py,
// relative error below 7.2e-15); e = exp(-x^2) is passed in.
__device__ inline double rcp_f64(double a);
template <bool TABLE>
__device__ inline double erfc_scaled_f64(double x) {
  const double s = fma(2.0, rcp_f64(fma(0.5, x, 1.0)), -1.0);
  return horner_f64<TABLE>(kErfcxCoef, kErfcxTable, s);
}

// FP64 building blocks of the pair scalar: hardware reciprocal and
// reciprocal-square-root estimates refined by two Newton steps each (the
// error of the estimate squares at every step: a few ulp after two), and
// exp(x) for x <= 0 by x = k ln2 + t, |t| <= ln2/2 (ln2 split into a head
// with 21 trailing zero bits, so k * head is exact, and a tail), the Taylor
// series of e^t to degree 14 (remainder below 1e-17) and a scaling by 2^k.
__device__ inline double rcp_f64(double a) {
  double y = __builtin_amdgcn_rcp(a);
  double e = fma(-a, y, 1.0);
  y = fma(y, e, y);
  e = fma(-a, y, 1.0);
  return fma(y, e, y);
}
__device__ inline double rsqrt_f64(double a) {
  double y = __builtin_amdgcn_rsq(a);
  // y <- y + y (1 - a y^2) / 2
  double e = fma(-a * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-a * y, y, 1.0);
  return fma(0.5 * y, e, y);
}
template <bool TABLE>
__device__ inline double exp_nonpos_f64(double x) {
  const double k = rint(x * 1.4426950408889634);
  double t = fma(-k, 0.6931471803691238, x);
  t = fma(-k, 1.9082149292705877e-10, t);
  return ldexp(horner_f64<TABLE>(kExpCoef, kExpTable, t), (int)k);
}

template <bool TABLE = false>
__device__ inline double pair_scalar_f64(const PairParams &pp, double r2, double qi, double qj) {
  const double rinv = rsqrt_f64(r2);
  const double inv_r2 = rinv * rinv;
  double f = 0.0;
  if (pp.do_coul && r2 <= pp.rc2 && qi != 0.0 && qj != 0.0) {
    const double r = r2 * rinv;
    const double e = exp_nonpos_f64<TABLE>(-pp.alpha * r2);
    const double R = erfc_scaled_f64<TABLE>(pp.sqrt_alpha * r);
    // G = erfc(x)/r^3 + 2 sqrt(a) e/(sqrt(pi) r^2) = e/r^2 (R/r + 2 sqrt(a)/sqrt(pi))
    const double G = e * inv_r2 * fma(R, rinv, pp.two_sqrt_alpha_over_sqrt_pi);
    f = pp.kc * qi * qj * G;
  }
  if (pp.do_lj && r2 <= pp.rlj2) {
    const double s2 = pp.sig2 * inv_r2;
    const double s6 = s2 * s2 * s2;
    f = fma(pp.eps24 * (2.0 * s6 * s6 - s6), inv_r2, f);
  }
  return f;
}

// FP32 form of the pair scalar: erfc(x) = exp(-x^2) R(x), R(x) = erfc(x) e^{x^2}
// as a degree-9 polynomial in t = 1/(1 + x/2) (fit over x in [0, 8] by
// fit_erfcx.py; relative error of the FP32 evaluation below 3.3e-7). The
// exponential exp(-alpha r^2) is shared with the second term of G.

__device__ inline float erfcx_poly(float t) {
  float r = -5.023304369e-02f;
  r = fmaf(r, t, 2.383836403e-01f);
  r = fmaf(r, t, -3.831243495e-01f);
  r = fmaf(r, t, 1.457629880e-01f);
  r = fmaf(r, t, 7.766769416e-02f);
  r = fmaf(r, t, 1.499599762e-01f);
  r = fmaf(r, t, 2.601579210e-01f);
  r = fmaf(r, t, 2.789792283e-01f);
  r = fmaf(r, t, 2.824637353e-01f);
  r = fmaf(r, t, -1.781403551e-05f);
  return r;
}

__device__ inline float pair_scalar_f32(const PairParams &pp, const PairF32 &pf, double r2d, float qiqj) {
  const float r2 = (float)r2d;
  const float rinv = __builtin_amdgcn_rsqf(r2);
  const float rinv2 = rinv * rinv;
  float f = 0.f;
  if (pp.do_coul && r2d <= pp.rc2 && qiqj != 0.f) {
    const float r = r2 * rinv;
    const float x = pf.sqrt_alpha * r;
    const float e = __builtin_amdgcn_exp2f(pf.neg_alpha_log2e * r2);
    const float t = __builtin_amdgcn_rcpf(fmaf(0.5f, x, 1.0f));
    const float erfc_x = e * erfcx_poly(t);
    const float G = fmaf(erfc_x * rinv, rinv2, pf.two_sqrt_alpha_over_sqrt_pi * e * rinv2);
    f = pf.kc * qiqj * G;
  }
  if (pp.do_lj && r2d <= pp.rlj2) {
    const float s2 = pf.sig2 * rinv2;
    const float s6 = s2 * s2 * s2;
    f = fmaf(pf.eps24 * fmaf(2.0f, s6 * s6, -s6), rinv2, f);
  }
  return f;
}

__device__ inline double pair_scalar_lj_f64(const PairParams &pp, double r2) {
  if (!(pp.do_lj && r2 <= pp.rlj2)) return 0.0;
  const double inv_r2 = rcp_f64(r2);
  const double s2 = pp.sig2 * inv_r2;
  const double s6 = s2 * s2 * s2;
  return pp.eps24 * (2.0 * s6 * s6 - s6) * inv_r2;
}

__device__ inline float pair_scalar_lj_f32(const PairParams &pp, const PairF32 &pf, double r2d) {
  if (!(pp.do_lj && r2d <= pp.rlj2)) return 0.f;
  const float rinv2 = __builtin_amdgcn_rcpf((float)r2d);
  const float s2 = pf.sig2 * rinv2;
  const float s6 = s2 * s2 * s2;
  return pf.eps24 * fmaf(2.0f, s6 * s6, -s6) * rinv2;
}

// Kahan-compensated FP32 accumulation of a 3-vector.
struct Kahan3 {
  float s[3] = {0.f, 0.f, 0.f}, c[3] = {0.f, 0.f, 0.f};
  __device__ inline void add(int k, float v) {
#pragma clang fp contract(off)
    const float y = v - c[k];
    const float t = s[k] + y;
    c[k] = (t - s[k]) - y;
    s[k] = t;
  }
  // s += a b with the product fused into the compensation step
  __device__ inline void add_prod(int k, float a, float b) {
#pragma clang fp contract(off)
    const float y = fmaf(a, b, -c[k]);
    const float t = s[k] + y;
    c[k] = (t - s[k]) - y;
    s[k] = t;
  }
  __device__ inline double get(int k) const { return (double)s[k] - (double)c[k]; }
};

__device__ inline double sq_dist(double dx, double dy, double dz) {
#pragma clang fp contract(off)
  return dx * dx + dy * dy + dz * dz;
}

__device__ inline double min_image(double a, double L) {
#pragma clang fp contract(off)
  return a - L * rint(a / L);
}

// Calls fn(jofs + j, p_j, id_j, shx, shy, shz) for the records j0..j1-1 of xq
// (and ids when WITH_ID, else id_j = 0); jofs separates the index ranges of
// natives (0) and ghosts (n). Four fixed slots: slot k holds record
// j + k and is reloaded with j + k + 4 right after use, so each load has
// three candidates of work to complete behind it. The lookahead reads up to
// kScanPad - 1 records past j1: every array scanned here is allocated with
// kScanPad records of padding, so those loads stay inside the allocation
// (their values are never used), and the addresses are plain increments.
template <bool WITH_ID, class Fn>
__device__ inline void scan_range(const double4 *__restrict__ xq, const int32_t *__restrict__ ids, int j0, int j1,
                                  double shx, double shy, double shz, Fn &&fn, int jofs = 0) {
  if (j0 >= j1) return;
  const double4 *p = xq + j0;
  const int32_t *q = WITH_ID ? ids + j0 : ids;
  double4 r0 = p[0], r1 = p[1], r2 = p[2], r3 = p[3];
  int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
  if (WITH_ID) {
    d0 = q[0];
    d1 = q[1];
    d2 = q[2];
    d3 = q[3];
  }
#pragma unroll 1
  for (int j = j0; j < j1; j += 4) {
    fn(jofs + j, r0, d0, shx, shy, shz);
    r0 = p[4];
    if (WITH_ID) d0 = q[4];
    if (j + 1 < j1) fn(jofs + j + 1, r1, d1, shx, shy, shz);
    r1 = p[5];
    if (WITH_ID) d1 = q[5];
    if (j + 2 < j1) fn(jofs + j + 2, r2, d2, shx, shy, shz);
    r2 = p[6];
    if (WITH_ID) d2 = q[6];
    if (j + 3 < j1) fn(jofs + j + 3, r3, d3, shx, shy, shz);
    r3 = p[7];
    if (WITH_ID) d3 = q[7];
    p += 4;
    if (WITH_ID) q += 4;
  }
}

// Walking particle of a thread-form traversal: position and the squared
// reach of the walk. Each stencil row is trimmed to the x-cells the reach
// sphere can touch: the gap g from (y, z) to the row's y/z cell slabs bounds
// the x extent by sqrt(r^2 - g^2), and rows with g > r are skipped. The
// gaps are shrunk and the extent grown by kTrimMargin, which covers the
// rounding of the binning (a particle binned to cell c lies within a few ulp
// of [c h, (c + 1) h]); every pair is still classified exactly afterwards.
struct Reach {
  double x, y, z, r2;
};
constexpr double kTrimMargin = 1e-9;
// Distance from p to the cell slab [c h, (c + 1) h] (unwrapped cell index c),
// minus the margin, at least 0.
__device__ inline double slab_gap(double p, int c, double h) {
#pragma clang fp contract(off)
  const double lo = (double)c * h, hi = lo + h;
  const double d = lo - p > 0.0 ? lo - p : (p - hi > 0.0 ? p - hi : 0.0);
  return d > kTrimMargin ? d - kTrimMargin : 0.0;
}
// x-cell range [*xa, *xb] (unwrapped, inside [cx - s, cx + s]) of a row at
// y/z gaps gy, gz; false if the row is out of reach.
__device__ inline bool row_range(const Grid &g, const Reach &R, double gy, double gz, int cx, int s, int *xa,
                                 int *xb) {
#pragma clang fp contract(off)
  const double rem = R.r2 - (gy * gy + gz * gz);
  if (rem < 0.0) return false;
  const double ext = sqrt(rem) + kTrimMargin;
  const int lo = (int)floor((R.x - ext) * g.inv_h[0]);
  const int hi = (int)floor((R.x + ext) * g.inv_h[0]);
  *xa = max(cx - s, lo);
  *xb = min(cx + s, hi);
  return *xa <= *xb;
}

// Periodic traversal: every particle j of species block `blk` in the
// (2 s.x + 1)(2 s.y + 1)(2 s.z + 1) cells around (cx, cy, cz) that the reach
// of R can touch;
// (shx, shy, shz) is the image shift of j (its image lies at r_j + shift).
// row_end() is called after each stencil row (the FP32C accumulators close a
// row's plain partial sum there).
struct NoRowEnd {
  __device__ inline void operator()() const {}
};
template <bool WITH_ID, class Fn, class RowEnd = NoRowEnd>
__device__ inline void for_stencil(const Grid &g, const int32_t *__restrict__ cell_start,
                                   const double4 *__restrict__ xq, const int32_t *__restrict__ ids, int blk, int cx,
                                   int cy, int cz, const Sten &s, const Reach &R, Fn &&fn, int64_t cell_base = 0,
                                   RowEnd row_end = RowEnd()) {
  const int64_t base = cell_base + (int64_t)blk * g.ncell;
  const double hy = g.L[1] / g.ny, hz = g.L[2] / g.nz;
  for (int oz = -s.z; oz <= s.z; ++oz) {
    const int az = cz + oz;
    const double gz = slab_gap(R.z, az, hz);
    if (gz * gz > R.r2) continue;
    const int qz = floor_div(az, g.nz);
    const int wz = az - qz * g.nz;
    const double shz = (double)qz * g.L[2];
    for (int oy = -s.y; oy <= s.y; ++oy) {
      const int ay = cy + oy;
      int a, a_end;
      if (!row_range(g, R, slab_gap(R.y, ay, hy), gz, cx, s.x, &a, &a_end)) continue;
      const int qy = floor_div(ay, g.ny);
      const int wy = ay - qy * g.ny;
      const double shy = (double)qy * g.L[1];
      const int64_t row = base + (int64_t)(wz * g.ny + wy) * g.nx;
      while (a <= a_end) {
        const int qx = floor_div(a, g.nx);
        const int b = min(a_end, (qx + 1) * g.nx - 1);
        const int j0 = cell_start[row + (a - qx * g.nx)];
        const int j1 = cell_start[row + (b - qx * g.nx) + 1];
        scan_range<WITH_ID>(xq, ids, j0, j1, (double)qx * g.L[0], shy, shz, fn);
        a = b + 1;
      }
      row_end();
    }
  }
}

// Ghost-shell traversal (no periodic images): the natives of the stencil
// rows that lie inside the native grid, then the ghosts of the same rows of
// the padded grid, each row trimmed to the reach of R. (cx, cy, cz) is a
// native cell. Ghosts reach fn with indices offset by nnat.
template <bool WITH_ID, class Fn, class RowEnd = NoRowEnd>
__device__ inline void for_stencil_ghost(const Grid &g, const int32_t *__restrict__ cell_start,
                                         const double4 *__restrict__ xq, const int32_t *__restrict__ ids,
                                         const int32_t *__restrict__ gcell_start, const double4 *__restrict__ gxq,
                                         const int32_t *__restrict__ gid, int nnat, int blk, int cx, int cy,
                                         int cz, const Sten &s, const Reach &R, Fn &&fn,
                                         RowEnd row_end = RowEnd()) {
  const int base = blk * g.ncell;
  const int pbase = blk * g.pncell;
  const double hy = g.L[1] / g.ny, hz = g.L[2] / g.nz;
  for (int oz = -s.z; oz <= s.z; ++oz) {
    const int z = cz + oz;
    const double gz = slab_gap(R.z, z, hz);
    if (gz * gz > R.r2) continue;
    for (int oy = -s.y; oy <= s.y; ++oy) {
      const int y = cy + oy;
      int xa, xb;
      if (!row_range(g, R, slab_gap(R.y, y, hy), gz, cx, s.x, &xa, &xb)) continue;
      const bool inner = z >= 0 && z < g.nz && y >= 0 && y < g.ny;
      if (inner) {
        const int na = max(xa, 0), nb = min(xb, g.nx - 1);
        if (na <= nb) {
          const int row = base + (z * g.ny + y) * g.nx;
          scan_range<WITH_ID>(xq, ids, cell_start[row + na], cell_start[row + nb + 1], 0.0, 0.0, 0.0, fn);
        }
      }
      // the padded cells over the native grid hold no ghosts: a row range
      // inside it has none to scan
      if (!inner || xa < 0 || xb >= g.nx) {
        const int prow = pbase + ((z + g.goff[2]) * g.pny + (y + g.goff[1])) * g.pnx + g.goff[0];
        scan_range<WITH_ID>(gxq, gid, gcell_start[prow + xa], gcell_start[prow + xb + 1], 0.0, 0.0, 0.0, fn, nnat);
      }
      row_end();
    }
  }
}

// Accumulator of the per-particle force in the two precision forms.
// add<true> evaluates Coulomb + LJ, add<false> LJ only (j neutral); TABLE
// selects the constant-memory polynomial coefficients (FP64 form).
template <bool F32>
struct ForceAcc;
template <>
struct ForceAcc<false> {
  double v[3] = {0.0, 0.0, 0.0};
  template <bool COUL, bool TABLE = false>
  __device__ inline void add(const PairParams &pp, const PairF32 &, double r2, double qi, double qj, double dx,
                             double dy, double dz) {
    const double sc = COUL ? pair_scalar_f64<TABLE>(pp, r2, qi, qj) : pair_scalar_lj_f64(pp, r2);
    v[0] = fma(sc, dx, v[0]);
    v[1] = fma(sc, dy, v[1]);
    v[2] = fma(sc, dz, v[2]);
  }
  __device__ inline double get(int k) const { return v[k]; }
  // the thread-form walks: same as add (FP64 sums need no row partials)
  template <bool COUL, bool TABLE = false>
  __device__ inline void add_row(const PairParams &pp, const PairF32 &pf, double r2, double qi, double qj, double dx,
                                 double dy, double dz) {
    add<COUL, TABLE>(pp, pf, r2, qi, qj, dx, dy, dz);
  }
  __device__ inline void flush_row() {}
};
template <>
struct ForceAcc<true> {
  Kahan3 k;
  float p[3] = {0.f, 0.f, 0.f};  // the current row's plain partial sums (add_row)
  // the thread-form walks: a row's terms summed plainly in FP32, the row sum
  // added with Kahan compensation at flush_row
  template <bool COUL, bool TABLE = false>
  __device__ inline void add_row(const PairParams &pp, const PairF32 &pf, double r2, double qi, double qj, double dx,
                                 double dy, double dz) {
    const float sc = COUL ? pair_scalar_f32(pp, pf, r2, (float)(qi * qj)) : pair_scalar_lj_f32(pp, pf, r2);
    p[0] = fmaf(sc, (float)dx, p[0]);
    p[1] = fmaf(sc, (float)dy, p[1]);
    p[2] = fmaf(sc, (float)dz, p[2]);
  }
  __device__ inline void flush_row() {
    for (int c = 0; c < 3; ++c) {
      k.add(c, p[c]);
      p[c] = 0.f;
    }
  }
  template <bool COUL, bool TABLE = false>
  __device__ inline void add(const PairParams &pp, const PairF32 &pf, double r2, double qi, double qj, double dx,
                             double dy, double dz) {
    const float sc = COUL ? pair_scalar_f32(pp, pf, r2, (float)(qi * qj)) : pair_scalar_lj_f32(pp, pf, r2);
    k.add_prod(0, sc, (float)dx);
    k.add_prod(1, sc, (float)dy);
    k.add_prod(2, sc, (float)dz);
  }
  __device__ inline double get(int c) const { return k.get(c); }
};

}  // namespace rbe

namespace rbe {

// ---------------------------------------------------------------------------
// Cluster traversal (8 x 8 lanes per wave)
// ---------------------------------------------------------------------------
// A wave computes the near field of a cluster of up to kCI consecutive
// particles of the cell order. Lane l plays i = cluster[l / kCJ] against the
// j-stream offset l % kCJ: the wave walks one shared sequence of candidate
// records kCJ at a time, so a load instruction touches kCJ consecutive
// records (two cache lines) and every lane runs the same loop. Particles of a
// cluster that lie in different cell rows (or species blocks, or replicas)
// are handled one row group after another; a group walks the union of its
// particles' stencils: the stencil rows around (cy, cz) with x running from
// min(cx) - s to max(cx) + s.
constexpr int kCI = 8;
constexpr int kCJ = 8;

// Buffer resource over `bytes` bytes at p (gfx9 raw buffer, no stride):
// loads that start past the end return zeros instead of touching memory.
__device__ inline __amdgpu_buffer_rsrc_t bounded_rsrc(const void *p, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, bytes, 0x00020000);
}
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
__device__ inline double dword_pair(uint32_t lo, uint32_t hi) {
  return __builtin_bit_cast(double, (uint64_t)lo | ((uint64_t)hi << 32));
}
// Record k of a segment (zeros past its end).
__device__ inline double4 load_record(__amdgpu_buffer_rsrc_t r, int k) {
  const u32x4 a = __builtin_amdgcn_raw_buffer_load_b128(r, k * 32, 0, 0);
  const u32x4 c = __builtin_amdgcn_raw_buffer_load_b128(r, k * 32 + 16, 0, 0);
  return make_double4(dword_pair(a.x, a.y), dword_pair(a.z, a.w), dword_pair(c.x, c.y), dword_pair(c.z, c.w));
}

// fn(ok, j, p_j, id_j, shx, shy, shz) for the records j0..j1-1 taken by this
// lane (j = jofs + j0 + b, jofs + j0 + b + kCJ, ...: jofs separates the index
// ranges of different arrays, natives 0 and ghosts n; ok = false on trips
// where this lane's record is past j1), one record prefetched ahead, then tick() once per trip with
// the whole wave. The trip count depends only on j0, j1, so the loop is the
// same for the wave; the segment is read through bounded buffer loads, so the
// lookahead needs no clamping.
template <bool WITH_ID, class Fn, class Tick>
__device__ inline void scan_cluster(const double4 *__restrict__ xq, const int32_t *__restrict__ ids, int j0, int j1,
                                    int b, double shx, double shy, double shz, Fn &&fn, Tick &&tick, int jofs = 0) {
  j0 = __builtin_amdgcn_readfirstlane(j0);  // uniform by construction; tell the compiler
  j1 = __builtin_amdgcn_readfirstlane(j1);
  if (j0 >= j1) return;
  const int cnt = j1 - j0;
  const __amdgpu_buffer_rsrc_t rx = bounded_rsrc(xq + j0, cnt * (int)sizeof(double4));
  const __amdgpu_buffer_rsrc_t ri = bounded_rsrc(WITH_ID ? ids + j0 : ids, WITH_ID ? cnt * 4 : 0);
  auto load_id = [&](int k) { return WITH_ID ? (int)__builtin_amdgcn_raw_buffer_load_b32(ri, k * 4, 0, 0) : 0; };
  int k = b;
  double4 r0 = load_record(rx, k);
  int d0 = load_id(k);
#pragma unroll 1
  for (int base = 0;; base += 2 * kCJ) {
    const double4 r1 = load_record(rx, k + kCJ);
    const int d1 = load_id(k + kCJ);
    fn(k < cnt, jofs + j0 + k, r0, d0, shx, shy, shz);
    tick();
    if (base + kCJ >= cnt) break;
    r0 = load_record(rx, k + 2 * kCJ);
    d0 = load_id(k + 2 * kCJ);
    fn(k + kCJ < cnt, jofs + j0 + k + kCJ, r1, d1, shx, shy, shz);
    tick();
    if (base + 2 * kCJ >= cnt) break;
    k += 2 * kCJ;
  }
}

// Row tables of a cluster walk: lane t of the wave resolves stencil row
// r0 + t (rows ordered z-major) into the cell-table bounds of its segments,
// so the cell-table loads of up to 64 rows are in flight together instead of
// one dependent pair per row; the walk then takes each row's bounds from its
// lane (wave-uniform reads).
struct RowSegs {
  int j0a, j1a, j0b, j1b;  // up to two segments of the row
  int qxa, qxb, qy, qz;    // their image shifts in boxes
};
__device__ inline RowSegs row_segs_at(const RowSegs &v, int k) {
  RowSegs u;
  u.j0a = __builtin_amdgcn_readlane(v.j0a, k);
  u.j1a = __builtin_amdgcn_readlane(v.j1a, k);
  u.j0b = __builtin_amdgcn_readlane(v.j0b, k);
  u.j1b = __builtin_amdgcn_readlane(v.j1b, k);
  u.qxa = __builtin_amdgcn_readlane(v.qxa, k);
  u.qxb = __builtin_amdgcn_readlane(v.qxb, k);
  u.qy = __builtin_amdgcn_readlane(v.qy, k);
  u.qz = __builtin_amdgcn_readlane(v.qz, k);
  return u;
}

// Periodic walk of species block `blk` (keys base + blk * C + cell) for a row
// group: rows (cy + oy, cz + oz), |oy| <= s.y, |oz| <= s.z, x from xa - s.x
// to xb + s.x, each row split where it crosses the periodic boundary (a cell
// met twice is met with two different image shifts, so no image is counted
// twice).
template <bool WITH_ID, class Fn, class Tick>
__device__ inline void cluster_walk(const Grid &g, const int32_t *__restrict__ cell_start,
                                    const double4 *__restrict__ xq, const int32_t *__restrict__ ids, int64_t base,
                                    int xa, int xb, int cy, int cz, const Sten &s, int b, Fn &&fn,
                                    Tick &&tick) {
  const int x0 = xa - s.x, x1 = xb + s.x;
  if (x1 - x0 + 1 > g.nx) {
    // the range wraps more than once (boxes of few cells): row by row
    for (int oz = -s.z; oz <= s.z; ++oz) {
      const int az = cz + oz;
      const int qz = floor_div(az, g.nz);
      const double shz = (double)qz * g.L[2];
      for (int oy = -s.y; oy <= s.y; ++oy) {
        const int ay = cy + oy;
        const int qy = floor_div(ay, g.ny);
        const double shy = (double)qy * g.L[1];
        const int64_t row = base + (int64_t)((az - qz * g.nz) * g.ny + (ay - qy * g.ny)) * g.nx;
        int x = x0;
        while (x <= x1) {
          const int qx = floor_div(x, g.nx);
          const int xe = min(x1, (qx + 1) * g.nx - 1);
          const int j0 = cell_start[row + (x - qx * g.nx)];
          const int j1 = cell_start[row + (xe - qx * g.nx) + 1];
          scan_cluster<WITH_ID>(xq, ids, j0, j1, b, (double)qx * g.L[0], shy, shz, fn, tick);
          x = xe + 1;
        }
      }
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  const int nyr = 2 * s.y + 1, nrows = nyr * (2 * s.z + 1);
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    RowSegs v{0, 0, 0, 0, 0, 0, 0, 0};
    const int r = r0 + lane;
    if (r < nrows) {
      const int az = cz + r / nyr - s.z, ay = cy + r % nyr - s.y;
      v.qz = floor_div(az, g.nz);
      v.qy = floor_div(ay, g.ny);
      const int64_t row = base + (int64_t)((az - v.qz * g.nz) * g.ny + (ay - v.qy * g.ny)) * g.nx;
      v.qxa = floor_div(x0, g.nx);
      const int ea = min(x1, (v.qxa + 1) * g.nx - 1);
      v.j0a = cell_start[row + (x0 - v.qxa * g.nx)];
      v.j1a = cell_start[row + (ea - v.qxa * g.nx) + 1];
      if (ea < x1) {  // wraps once: the rest lies in the next image
        v.qxb = v.qxa + 1;
        v.j0b = cell_start[row];
        v.j1b = cell_start[row + (x1 - v.qxb * g.nx) + 1];
      }
    }
    const int nr = min(64, nrows - r0);
    for (int k = 0; k < nr; ++k) {
      const RowSegs u = row_segs_at(v, k);
      const double shy = (double)u.qy * g.L[1], shz = (double)u.qz * g.L[2];
      scan_cluster<WITH_ID>(xq, ids, u.j0a, u.j1a, b, (double)u.qxa * g.L[0], shy, shz, fn, tick);
      scan_cluster<WITH_ID>(xq, ids, u.j0b, u.j1b, b, (double)u.qxb * g.L[0], shy, shz, fn, tick);
    }
  }
}

// Ghost-shell walk (no periodic images): the native part of each stencil row
// clipped to the native grid, then the same row of the padded ghost grid
// (row tables as in the periodic walk: segment a native, segment b ghost).
// Ghost records are passed to fn with indices offset by nnat, so no ghost
// index equals a native one.
template <bool WITH_ID, class Fn, class Tick>
__device__ inline void cluster_walk_ghost(const Grid &g, const int32_t *__restrict__ cell_start,
                                          const double4 *__restrict__ xq, const int32_t *__restrict__ ids,
                                          const int32_t *__restrict__ gcell_start, const double4 *__restrict__ gxq,
                                          const int32_t *__restrict__ gid, int nnat, int blk, int xa, int xb,
                                          int cy, int cz, const Sten &s, int b, Fn &&fn, Tick &&tick) {
  const int64_t base = (int64_t)blk * g.ncell;
  const int64_t pbase = (int64_t)blk * g.pncell;
  const int na = max(xa - s.x, 0), nb = min(xb + s.x, g.nx - 1);
  const int lane = threadIdx.x & 63;
  const int nyr = 2 * s.y + 1, nrows = nyr * (2 * s.z + 1);
  for (int r0 = 0; r0 < nrows; r0 += 64) {
    RowSegs v{0, 0, 0, 0, 0, 0, 0, 0};
    const int r = r0 + lane;
    if (r < nrows) {
      const int z = cz + r / nyr - s.z, y = cy + r % nyr - s.y;
      if (z >= 0 && z < g.nz && y >= 0 && y < g.ny) {
        const int64_t row = base + (int64_t)(z * g.ny + y) * g.nx;
        v.j0a = cell_start[row + na];
        v.j1a = cell_start[row + nb + 1];
      }
      const int64_t prow = pbase + (int64_t)((z + g.goff[2]) * g.pny + (y + g.goff[1])) * g.pnx + g.goff[0];
      v.j0b = gcell_start[prow + xa - s.x];
      v.j1b = gcell_start[prow + xb + s.x + 1];
    }
    const int nr = min(64, nrows - r0);
    for (int k = 0; k < nr; ++k) {
      const RowSegs u = row_segs_at(v, k);
      scan_cluster<WITH_ID>(xq, ids, u.j0a, u.j1a, b, 0.0, 0.0, 0.0, fn, tick);
      scan_cluster<WITH_ID>(gxq, gid, u.j0b, u.j1b, b, 0.0, 0.0, 0.0, fn, tick, nnat);
    }
  }
}

// Row groups of a cluster wave. `valid`: this lane's i exists; rowkey: a
// value shared exactly by the particles of one cell row (and species block,
// and replica). Calls gfn(in, leader, xa, xb) once per distinct row, where
// `in` says whether this lane's i belongs to the group, `leader` is a lane of
// the group and [xa, xb] the group's x-cell range (all wave-uniform).
template <class GroupFn>
__device__ inline void for_each_row_group(bool valid, int64_t rowkey, int cx, GroupFn &&gfn) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(valid && (lane % kCJ) == 0);
  while (todo) {
    const int leader = __builtin_amdgcn_readfirstlane(__ffsll((long long)todo) - 1);
    const int64_t R = __shfl(rowkey, leader, 64);
    const bool in = valid && rowkey == R;
    int xa = in ? cx : 0x7FFFFFFF, xb = in ? cx : -0x7FFFFFFF;
#pragma unroll
    for (int o = kCJ; o < 64; o <<= 1) {
      xa = min(xa, __shfl_xor(xa, o, 64));
      xb = max(xb, __shfl_xor(xb, o, 64));
    }
    xa = __builtin_amdgcn_readfirstlane(xa);
    xb = __builtin_amdgcn_readfirstlane(xb);
    gfn(in, leader, xa, xb);
    todo &= ~__ballot(in && (lane % kCJ) == 0);
  }
}

// Sum over the kCJ lanes that share an i (fixed order: deterministic).
__device__ inline double sum_j_lanes(double v) {
#pragma unroll
  for (int o = 1; o < kCJ; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline int sum_j_lanes(int v) {
#pragma unroll
  for (int o = 1; o < kCJ; o <<= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace rbe
