// Near-field force (Sec. 2.1, Eq. 7-8, 10-11): erfc-screened Coulomb plus
// 12-6 Lennard-Jones over a cell list, with the core-shell random batch list.
//
// One thread per particle i (cell order), full neighbour sums, no atomics.
// A thread walks the stencil of cells around its own cell; a stencil row is
// a run of consecutive x-cells, contiguous in the sorted arrays, split only
// where it crosses the periodic boundary (each piece carries the image shift
// that the minimum-image convention assigns to it).
//
// Species blocks: charged particles occupy keys [0, C), neutral ones
// [C, 2C). Coulomb terms only involve charged pairs, so without the random
// batch list a charged i walks the charged block out to r_coul and the
// neutral block out to r_lj; a neutral i walks both blocks out to r_lj.
//
// Random batch list (Eq. 10-11), for particles whose shell terms can be
// non-zero: every j within r_coul is classified with the squared distance
// computed without contraction (the same IEEE expression as the CPU oracle):
// core (r^2 <= r_core^2) terms are summed exactly; shell members are counted
// and their ranking keys kept in a sorted register list of the 32 smallest.
// The batch is the p smallest keys (all members if #S <= p); a key maps back
// to the particle id (the key is a bijection of id_j), the id to its sorted
// slot, and the batch terms are summed with the weight #S/|B|.
//
// Pair force on i: (kc q_i q_j G(r) + G_LJ(r)) d, d = r_i - r_j,
//   G(r)    = erfc(sqrt(a) r)/r^3 + 2 sqrt(a) exp(-a r^2)/(sqrt(pi) r^2),
//   G_LJ(r) = 24 eps (2 sigma^12/r^14 - sigma^6/r^8).
#include "kernels.h"

namespace rbe {

// FP64 erfc(x) = exp(-x^2) R(x) with R(x) = erfc(x) e^{x^2} a degree-20
// polynomial in s = 2/(1 + x/2) - 1 (fit over x in [0, 8] by fit_erfcx.py,
// relative error below 7.2e-15); e = exp(-x^2) is passed in.
__device__ inline double erfc_scaled_f64(double x) {
  const double s = 2.0 / fma(0.5, x, 1.0) - 1.0;
  double r = 1.63618628481317543e-08;
  r = fma(r, s, -4.60928758649811430e-08);
  r = fma(r, s, -6.88442333452307132e-08);
  r = fma(r, s, 4.40190654889049080e-07);
  r = fma(r, s, -4.46917185831068957e-07);
  r = fma(r, s, -1.14063358111397811e-06);
  r = fma(r, s, 3.75537844601685302e-06);
  r = fma(r, s, -1.41703053499259700e-06);
  r = fma(r, s, -1.39602653735770222e-05);
  r = fma(r, s, 2.75867068654632672e-05);
  r = fma(r, s, 2.75241444094816018e-05);
  r = fma(r, s, -1.74362281120596591e-04);
  r = fma(r, s, 4.35557661104548185e-05);
  r = fma(r, s, 9.81977137355043118e-04);
  r = fma(r, s, -8.47143262890503600e-04);
  r = fma(r, s, -6.99746174546772310e-03);
  r = fma(r, s, 3.73289240473987467e-03);
  r = fma(r, s, 7.89785810158994406e-02);
  r = fma(r, s, 2.41658194242463487e-01);
  r = fma(r, s, 4.27185847413955655e-01);
  r = fma(r, s, 2.55395676310504194e-01);
  return r;
}

__device__ inline double pair_scalar_f64(const PairParams &pp, double r2, double qi, double qj) {
  const double inv_r2 = 1.0 / r2;
  double f = 0.0;
  if (pp.do_coul && r2 <= pp.rc2 && qi != 0.0 && qj != 0.0) {
    const double r = sqrt(r2);
    const double e = exp(-pp.alpha * r2);
    const double R = erfc_scaled_f64(pp.sqrt_alpha * r);
    // G = erfc(x)/r^3 + 2 sqrt(a) e/(sqrt(pi) r^2) = e/r^2 (R/r + 2 sqrt(a)/sqrt(pi))
    const double G = e * inv_r2 * (R / r + pp.two_sqrt_alpha_over_sqrt_pi);
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
struct PairF32 {
  float sqrt_alpha, neg_alpha_log2e, two_sqrt_alpha_over_sqrt_pi, kc, eps24, sig2;
};

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
  const double inv_r2 = 1.0 / r2;
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

// Calls fn(j, p_j, id_j, shx, shy, shz) for the records j0..j1-1 of xq (and
// ids when WITH_ID, else id_j = 0). Four fixed slots: slot k holds record
// j + k and is reloaded with j + k + 4 right after use, so each load has
// three candidates of work to complete behind it. Indices past the range are
// clamped to its last record (always a valid address).
template <bool WITH_ID, class Fn>
__device__ inline void scan_range(const double4 *__restrict__ xq, const int32_t *__restrict__ ids, int j0, int j1,
                                  double shx, double shy, double shz, Fn &&fn) {
  if (j0 >= j1) return;
  const int last = j1 - 1;
  double4 r0 = xq[j0], r1 = xq[min(j0 + 1, last)], r2 = xq[min(j0 + 2, last)], r3 = xq[min(j0 + 3, last)];
  int d0 = 0, d1 = 0, d2 = 0, d3 = 0;
  if (WITH_ID) {
    d0 = ids[j0];
    d1 = ids[min(j0 + 1, last)];
    d2 = ids[min(j0 + 2, last)];
    d3 = ids[min(j0 + 3, last)];
  }
#pragma unroll 1
  for (int j = j0; j < j1; j += 4) {
    fn(j, r0, d0, shx, shy, shz);
    r0 = xq[min(j + 4, last)];
    if (WITH_ID) d0 = ids[min(j + 4, last)];
    if (j + 1 < j1) fn(j + 1, r1, d1, shx, shy, shz);
    r1 = xq[min(j + 5, last)];
    if (WITH_ID) d1 = ids[min(j + 5, last)];
    if (j + 2 < j1) fn(j + 2, r2, d2, shx, shy, shz);
    r2 = xq[min(j + 6, last)];
    if (WITH_ID) d2 = ids[min(j + 6, last)];
    if (j + 3 < j1) fn(j + 3, r3, d3, shx, shy, shz);
    r3 = xq[min(j + 7, last)];
    if (WITH_ID) d3 = ids[min(j + 7, last)];
  }
}

// Periodic traversal: every particle j of species block `blk` in the
// (2s+1)^3 cells around (cx, cy, cz); (shx, shy, shz) is the image shift of j
// (its image lies at r_j + shift).
template <bool WITH_ID, class Fn>
__device__ inline void for_stencil(const Grid &g, const int32_t *__restrict__ cell_start,
                                   const double4 *__restrict__ xq, const int32_t *__restrict__ ids, int blk, int cx,
                                   int cy, int cz, int s, Fn &&fn) {
  const int base = blk * g.ncell;
  for (int oz = -s; oz <= s; ++oz) {
    const int az = cz + oz;
    const int qz = floor_div(az, g.nz);
    const int wz = az - qz * g.nz;
    const double shz = (double)qz * g.L[2];
    for (int oy = -s; oy <= s; ++oy) {
      const int ay = cy + oy;
      const int qy = floor_div(ay, g.ny);
      const int wy = ay - qy * g.ny;
      const double shy = (double)qy * g.L[1];
      const int row = base + (wz * g.ny + wy) * g.nx;
      int a = cx - s;
      const int a_end = cx + s;
      while (a <= a_end) {
        const int qx = floor_div(a, g.nx);
        const int b = min(a_end, (qx + 1) * g.nx - 1);
        const int j0 = cell_start[row + (a - qx * g.nx)];
        const int j1 = cell_start[row + (b - qx * g.nx) + 1];
        scan_range<WITH_ID>(xq, ids, j0, j1, (double)qx * g.L[0], shy, shz, fn);
        a = b + 1;
      }
    }
  }
}

// Ghost-shell traversal (no periodic images): the natives of the stencil
// rows that lie inside the native grid, then the ghosts of the same rows of
// the padded grid. (cx, cy, cz) is a native cell.
template <bool WITH_ID, class Fn>
__device__ inline void for_stencil_ghost(const Grid &g, const int32_t *__restrict__ cell_start,
                                         const double4 *__restrict__ xq, const int32_t *__restrict__ ids,
                                         const int32_t *__restrict__ gcell_start, const double4 *__restrict__ gxq,
                                         const int32_t *__restrict__ gid, int blk, int cx, int cy, int cz, int s,
                                         Fn &&fn) {
  const int base = blk * g.ncell;
  const int pbase = blk * g.pncell;
  const int xa = max(cx - s, 0), xb = min(cx + s, g.nx - 1);
  for (int oz = -s; oz <= s; ++oz) {
    const int z = cz + oz;
    for (int oy = -s; oy <= s; ++oy) {
      const int y = cy + oy;
      if (z >= 0 && z < g.nz && y >= 0 && y < g.ny) {
        const int row = base + (z * g.ny + y) * g.nx;
        scan_range<WITH_ID>(xq, ids, cell_start[row + xa], cell_start[row + xb + 1], 0.0, 0.0, 0.0, fn);
      }
      const int prow = pbase + ((z + g.goff[2]) * g.pny + (y + g.goff[1])) * g.pnx + g.goff[0];
      scan_range<WITH_ID>(gxq, gid, gcell_start[prow + cx - s], gcell_start[prow + cx + s + 1], 0.0, 0.0, 0.0, fn);
    }
  }
}

// Accumulator of the per-particle force in the two precision forms.
// add<true> evaluates Coulomb + LJ, add<false> LJ only (j neutral).
template <bool F32>
struct ForceAcc;
template <>
struct ForceAcc<false> {
  double v[3] = {0.0, 0.0, 0.0};
  template <bool COUL>
  __device__ inline void add(const PairParams &pp, const PairF32 &, double r2, double qi, double qj, double dx,
                             double dy, double dz) {
    const double sc = COUL ? pair_scalar_f64(pp, r2, qi, qj) : pair_scalar_lj_f64(pp, r2);
    v[0] = fma(sc, dx, v[0]);
    v[1] = fma(sc, dy, v[1]);
    v[2] = fma(sc, dz, v[2]);
  }
  __device__ inline double get(int k) const { return v[k]; }
};
template <>
struct ForceAcc<true> {
  Kahan3 k;
  template <bool COUL>
  __device__ inline void add(const PairParams &pp, const PairF32 &pf, double r2, double qi, double qj, double dx,
                             double dy, double dz) {
    const float sc = COUL ? pair_scalar_f32(pp, pf, r2, (float)(qi * qj)) : pair_scalar_lj_f32(pp, pf, r2);
    k.add(0, sc * (float)dx);
    k.add(1, sc * (float)dy);
    k.add(2, sc * (float)dz);
  }
  __device__ inline double get(int c) const { return k.get(c); }
};

struct PairCtx {
  PairParams pp;
  PairF32 pf;
  const double4 *__restrict__ xq;
  const int32_t *__restrict__ ids;
  const int32_t *__restrict__ cell_start;
  const int32_t *__restrict__ inv_id;
  double *__restrict__ fx;
  double *__restrict__ fy;
  double *__restrict__ fz;
  unsigned long long *__restrict__ counters;  // [4] when counting
  int64_t i0, i1;                             // particle range of this launch
  int64_t n;                                  // all particles
  // ghost shell (GHOST kernels only)
  const double4 *__restrict__ gxq;
  const int32_t *__restrict__ gid;
  const int32_t *__restrict__ gcell_start;
};

// Stencil walk of the right kind for the kernel.
template <bool GHOST, bool WITH_ID, class Fn>
__device__ inline void stencil(const PairCtx &c, int blk, int cx, int cy, int cz, int s, Fn &&fn) {
  if (GHOST)
    for_stencil_ghost<WITH_ID>(c.pp.g, c.cell_start, c.xq, c.ids, c.gcell_start, c.gxq, c.gid, blk, cx, cy, cz, s,
                               fn);
  else
    for_stencil<WITH_ID>(c.pp.g, c.cell_start, c.xq, c.ids, blk, cx, cy, cz, s, fn);
}

template <bool COUNT>
__device__ inline void flush_counts(const PairCtx &c, unsigned long long n_coul, unsigned long long n_lj,
                                    unsigned long long n_tested, unsigned long long n_shell) {
  if (COUNT) {
    atomicAdd(&c.counters[0], n_coul);
    atomicAdd(&c.counters[1], n_lj);
    atomicAdd(&c.counters[2], n_tested);
    atomicAdd(&c.counters[3], n_shell);
  }
}

// Plain cutoff sums for particle i. MODE 0: neutral i (LJ over both species
// blocks out to r_lj); MODE 1: charged i (charged block out to
// max(r_coul, r_lj), neutral block out to r_lj).
template <bool F32, bool COUNT, int MODE, bool GHOST>
__global__ void __launch_bounds__(256) k_pair_plain(PairCtx c) {
  const int64_t i = c.i0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= c.i1) return;
  const PairParams &pp = c.pp;
  const Grid &g = pp.g;
  const double4 pi4 = c.xq[i];
  const double xi = pi4.x, yi = pi4.y, zi = pi4.z, qi = pi4.w;
  const int cx = cell_coord(xi, g.inv_h[0], g.nx);
  const int cy = cell_coord(yi, g.inv_h[1], g.ny);
  const int cz = cell_coord(zi, g.inv_h[2], g.nz);
  ForceAcc<F32> acc;
  unsigned long long n_coul = 0, n_lj = 0, n_tested = 0;
  // Coulomb + LJ against charged j (block 0 of a charged i)
  auto visit_q = [&](int j, const double4 &pj, int, double shx, double shy, double shz) {
    const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (COUNT) ++n_tested;
    if (r2 == 0.0 && j == (int)i) return;
    if (r2 <= pp.rc2 || r2 <= pp.rlj2) {
      acc.template add<true>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
      if (COUNT) {
        n_coul += (pp.do_coul && r2 <= pp.rc2);
        n_lj += (pp.do_lj && r2 <= pp.rlj2);
      }
    }
  };
  // LJ only (every other species pairing)
  auto visit_lj = [&](int j, const double4 &pj, int, double shx, double shy, double shz) {
    const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (COUNT) ++n_tested;
    if (r2 == 0.0 && j == (int)i) return;
    if (r2 <= pp.rlj2) {
      acc.template add<false>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
      if (COUNT) n_lj += pp.do_lj;
    }
  };
  if (MODE == 1) {
    stencil<GHOST, false>(c, 0, cx, cy, cz, pp.s_coul, visit_q);
    if (pp.do_lj) stencil<GHOST, false>(c, 1, cx, cy, cz, pp.s_lj, visit_lj);
  } else if (pp.do_lj) {
    stencil<GHOST, false>(c, 0, cx, cy, cz, pp.s_lj, visit_lj);
    stencil<GHOST, false>(c, 1, cx, cy, cz, pp.s_lj, visit_lj);
  }
  c.fx[i] = acc.get(0);
  c.fy[i] = acc.get(1);
  c.fz[i] = acc.get(2);
  flush_counts<COUNT>(c, n_coul, n_lj, n_tested, 0);
}

// Sorted insertion of k into the ascending list L[0..CAP), dropping the
// largest: the new L[t] is the (t+1)-th smallest of L and k, which is
// min(L[t], max(L[t-1], k)); walking t downwards updates L in place.
template <int CAP>
__device__ inline void sorted_insert(uint32_t (&L)[CAP], uint32_t k) {
#pragma unroll
  for (int t = CAP - 1; t > 0; --t) L[t] = min(L[t], max(L[t - 1], k));
  L[0] = min(L[0], k);
}

// Random batch list (Eq. 10-11) for particle i: exact core, ranked shell.
// CAP >= p slots hold the smallest shell keys in ascending order.
template <bool F32, bool COUNT, int CAP, bool GHOST>
__global__ void __launch_bounds__(256) k_pair_rbl(PairCtx c) {
  const int64_t i = c.i0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= c.i1) return;
  const PairParams &pp = c.pp;
  const Grid &g = pp.g;
  const double4 pi4 = c.xq[i];
  const double xi = pi4.x, yi = pi4.y, zi = pi4.z, qi = pi4.w;
  const int cx = cell_coord(xi, g.inv_h[0], g.nx);
  const int cy = cell_coord(yi, g.inv_h[1], g.ny);
  const int cz = cell_coord(zi, g.inv_h[2], g.nz);
  ForceAcc<F32> acc;
  unsigned long long n_coul = 0, n_lj = 0, n_tested = 0;
  uint32_t keys[CAP];
#pragma unroll
  for (int t = 0; t < CAP; ++t) keys[t] = 0xFFFFFFFFu;
  const ShellKey sk = shell_key_of(pp.shell_key, c.ids[i]);
  int ns = 0;
  auto visit = [&](int j, const double4 &pj, int idj, double shx, double shy, double shz) {
    const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (COUNT) ++n_tested;
    if (r2 == 0.0 && j == (int)i) return;
    if (r2 <= pp.rcore2) {
      acc.template add<true>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
      if (COUNT) {
        n_coul += (pp.do_coul && qi != 0.0 && pj.w != 0.0);
        n_lj += (pp.do_lj && r2 <= pp.rlj2);
      }
    } else if (r2 <= pp.rc2) {
      ++ns;
      const uint32_t k = shell_rank(sk, idj);
      if (k < keys[CAP - 1]) sorted_insert<CAP>(keys, k);
    }
  };
  stencil<GHOST, true>(c, 0, cx, cy, cz, pp.s_coul, visit);
  stencil<GHOST, true>(c, 1, cx, cy, cz, pp.s_coul, visit);
  double f0 = acc.get(0), f1 = acc.get(1), f2 = acc.get(2);
  if (ns > 0) {
    const int nb = ns < pp.p_shell ? ns : pp.p_shell;
    ForceAcc<F32> sh;
#pragma unroll
    for (int t = 0; t < CAP; ++t) {
      if (t < nb) {
        const int32_t idj = shell_id_of(sk, keys[t]);
        if ((uint32_t)idj >= (uint32_t)c.n) continue;  // bad ids (flagged by the inverse map)
        const int j = c.inv_id[idj];
        if ((uint32_t)j >= (uint32_t)c.n) continue;
        const double4 pj = c.xq[j];
        const double dx = min_image(xi - pj.x, g.L[0]);
        const double dy = min_image(yi - pj.y, g.L[1]);
        const double dz = min_image(zi - pj.z, g.L[2]);
        const double r2 = sq_dist(dx, dy, dz);
        sh.template add<true>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
        if (COUNT) {
          n_coul += (pp.do_coul && qi != 0.0 && pj.w != 0.0);
          n_lj += (pp.do_lj && r2 <= pp.rlj2);
        }
      }
    }
    const double scale = (double)ns / (double)nb;
    f0 = fma(scale, sh.get(0), f0);
    f1 = fma(scale, sh.get(1), f1);
    f2 = fma(scale, sh.get(2), f2);
  }
  c.fx[i] = f0;
  c.fy[i] = f1;
  c.fz[i] = f2;
  flush_counts<COUNT>(c, n_coul, n_lj, n_tested, (unsigned long long)ns);
}

constexpr int kShellThreads = 256;
constexpr int kShellRoom = 16;  // buffer slots beyond the batch capacity

// Shell part of the random batch list (Eq. 10-11) for a charged i whose core
// terms were summed by the plain kernel with the Coulomb cutoff set to r_core:
// every j with r_core^2 < r^2 <= r_coul^2 (same contraction-free r^2 as the
// core test) is counted and ranked; the p smallest keys form the batch, whose
// terms are added to f_i with the weight #S_i/|B_i|.
//
// Selection: each lane appends the keys below its threshold tau to its own
// LDS buffer (CAP + kShellRoom slots). When a buffer fills, the buffers of the
// wave are reduced to their p smallest keys and a full lane's tau becomes the
// largest of them: any later key above tau has p smaller keys before it and
// cannot be in the batch (keys are distinct). So a buffer always contains the
// p smallest keys its lane has seen.
template <bool F32, bool COUNT, int CAP, bool GHOST>
__global__ void __launch_bounds__(kShellThreads) k_pair_shell(PairCtx c) {
  constexpr int B = CAP + kShellRoom;
  __shared__ uint32_t sbuf[B * kShellThreads];
  const int tid = threadIdx.x;
  const int64_t i = c.i0 + blockIdx.x * (int64_t)blockDim.x + tid;
  if (i >= c.i1) return;
  const PairParams &pp = c.pp;
  const Grid &g = pp.g;
  const int p = pp.p_shell;
  const double4 pi4 = c.xq[i];
  const double xi = pi4.x, yi = pi4.y, zi = pi4.z, qi = pi4.w;
  const int cx = cell_coord(xi, g.inv_h[0], g.nx);
  const int cy = cell_coord(yi, g.inv_h[1], g.ny);
  const int cz = cell_coord(zi, g.inv_h[2], g.nz);
  const ShellKey sk = shell_key_of(pp.shell_key, c.ids[i]);
  int ns = 0, cnt = 0;
  int sorted = 0;  // buf[0..sorted) is ascending (left by the last reduction)
  uint32_t tau = 0xFFFFFFFFu;
  bool have_tau = false;
  unsigned long long n_tested = 0, n_coul = 0, n_lj = 0;
  // reduce the buffer to its min(p, cnt) smallest keys, sorted; returns them in L
  auto reduce = [&](uint32_t (&L)[CAP]) {
#pragma unroll
    for (int t = 0; t < CAP; ++t) L[t] = t < sorted ? sbuf[t * kShellThreads + tid] : 0xFFFFFFFFu;
    for (int t = sorted; t < cnt; ++t) sorted_insert<CAP>(L, sbuf[t * kShellThreads + tid]);
    const int keep = cnt < p ? cnt : p;
#pragma unroll
    for (int t = 0; t < CAP; ++t)
      if (t < keep) sbuf[t * kShellThreads + tid] = L[t];
    cnt = keep;
    sorted = keep;
  };
  auto visit = [&](int, const double4 &pj, int idj, double shx, double shy, double shz) {
    const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (COUNT) ++n_tested;
    if (r2 > pp.rcore2 && r2 <= pp.rc2) {
      ++ns;
      const uint32_t k = shell_rank(sk, idj);
      if (!have_tau || k < tau) sbuf[cnt++ * kShellThreads + tid] = k;
    }
    // every active lane reduces when one lane's buffer is full (one pass of
    // the wave instead of one per lane)
    if (__any(cnt == B)) {
      uint32_t L[CAP];
      reduce(L);
      if (cnt == p) {
#pragma unroll
        for (int t = 0; t < CAP; ++t)
          if (t == p - 1) tau = L[t];
        have_tau = true;
      }
    }
  };
  stencil<GHOST, true>(c, 0, cx, cy, cz, pp.s_coul, visit);
  stencil<GHOST, true>(c, 1, cx, cy, cz, pp.s_coul, visit);
  if (ns > 0) {
    uint32_t L[CAP];
    reduce(L);
    const int nb = cnt;  // = min(ns, p)
    ForceAcc<F32> sh;
#pragma unroll
    for (int t = 0; t < CAP; ++t) {
      if (t < nb) {
        const int32_t idj = shell_id_of(sk, L[t]);
        if ((uint32_t)idj >= (uint32_t)c.n) continue;  // bad ids (flagged by the inverse map)
        const int j = c.inv_id[idj];
        if ((uint32_t)j >= (uint32_t)c.n) continue;
        const double4 pj = c.xq[j];
        const double dx = min_image(xi - pj.x, g.L[0]);
        const double dy = min_image(yi - pj.y, g.L[1]);
        const double dz = min_image(zi - pj.z, g.L[2]);
        const double r2 = sq_dist(dx, dy, dz);
        sh.template add<true>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
        if (COUNT) {
          n_coul += (pp.do_coul && qi != 0.0 && pj.w != 0.0);
          n_lj += (pp.do_lj && r2 <= pp.rlj2);
        }
      }
    }
    const double scale = (double)ns / (double)nb;
    c.fx[i] = fma(scale, sh.get(0), c.fx[i]);
    c.fy[i] = fma(scale, sh.get(1), c.fy[i]);
    c.fz[i] = fma(scale, sh.get(2), c.fz[i]);
  }
  flush_counts<COUNT>(c, n_coul, n_lj, n_tested, (unsigned long long)ns);
}

static PairF32 make_f32(const PairParams &pp) {
  PairF32 pf;
  pf.sqrt_alpha = (float)pp.sqrt_alpha;
  pf.neg_alpha_log2e = (float)(-pp.alpha * 1.4426950408889634074);
  pf.two_sqrt_alpha_over_sqrt_pi = (float)pp.two_sqrt_alpha_over_sqrt_pi;
  pf.kc = (float)pp.kc;
  pf.eps24 = (float)pp.eps24;
  pf.sig2 = (float)pp.sig2;
  return pf;
}

template <class K>
static void launch_range(K kernel, PairCtx c, int64_t i0, int64_t i1, hipStream_t st) {
  if (i1 <= i0) return;
  c.i0 = i0;
  c.i1 = i1;
  const unsigned blocks = (unsigned)((i1 - i0 + 255) / 256);
  kernel<<<blocks, 256, 0, st>>>(c);
}

template <bool F32, bool COUNT, bool GHOST>
static void launch_rbl(PairCtx c, int64_t i0, int64_t i1, bool split, hipStream_t st) {
  const int p = c.pp.p_shell;
  if (split) {
    if (p <= 8) launch_range(k_pair_shell<F32, COUNT, 8, GHOST>, c, i0, i1, st);
    else if (p <= 16) launch_range(k_pair_shell<F32, COUNT, 16, GHOST>, c, i0, i1, st);
    else if (p <= 24) launch_range(k_pair_shell<F32, COUNT, 24, GHOST>, c, i0, i1, st);
    else launch_range(k_pair_shell<F32, COUNT, 32, GHOST>, c, i0, i1, st);
    return;
  }
  if (p <= 16) launch_range(k_pair_rbl<F32, COUNT, 16, GHOST>, c, i0, i1, st);
  else launch_range(k_pair_rbl<F32, COUNT, 32, GHOST>, c, i0, i1, st);
}

// Charged particles occupy [0, nq) of the sorted order, neutral ones [nq, n).
// With the random batch list and r_lj <= r_core, a charged particle's core is
// the plain sum with the Coulomb cutoff set to r_core (same r^2 test), and its
// shell is added by the shell kernel; otherwise one fused kernel does both.
// part: PAIR_PART_CHARGED, PAIR_PART_SHELL (after CHARGED) or PAIR_PART_NEUTRAL.
template <bool F32, bool COUNT, bool GHOST>
static void launch_part(PairCtx c, int64_t nq, int part, hipStream_t st) {
  const PairParams pp = c.pp;
  const bool split = pp.rbl && pp.rlj2 <= pp.rcore2;
  if (pp.rbl && !split) {
    if (part == PAIR_PART_CHARGED) launch_rbl<F32, COUNT, GHOST>(c, 0, c.n, false, st);
    return;
  }
  if (part == PAIR_PART_CHARGED) {
    PairCtx core = c;
    if (split) {
      core.pp.rc2 = pp.rcore2;
      core.pp.s_coul = pp.s_core;
    }
    launch_range(k_pair_plain<F32, COUNT, 1, GHOST>, core, 0, nq, st);
  } else if (part == PAIR_PART_SHELL) {
    if (split) launch_rbl<F32, COUNT, GHOST>(c, 0, nq, true, st);
  } else {
    launch_range(k_pair_plain<F32, COUNT, 0, GHOST>, c, nq, c.n, st);
  }
}

template <bool GHOST>
static void launch_prec(int prec, PairCtx c, int64_t nq, int part, hipStream_t st) {
  if (prec == RBE_FP32C) {
    if (c.counters) launch_part<true, true, GHOST>(c, nq, part, st);
    else launch_part<true, false, GHOST>(c, nq, part, st);
  } else {
    if (c.counters) launch_part<false, true, GHOST>(c, nq, part, st);
    else launch_part<false, false, GHOST>(c, nq, part, st);
  }
}

void launch_pair(int prec, int part, const PairParams &pp, int64_t n, int64_t nq, const Sorted &s,
                 const int32_t *cell_start, const int32_t *inv_id, const GhostBuffers *gb, double *fx, double *fy,
                 double *fz, PairCounters cnt, hipStream_t st) {
  if (n <= 0) return;
  PairCtx c;
  c.pp = pp;
  c.pf = make_f32(pp);
  c.xq = s.xq;
  c.ids = s.id;
  c.cell_start = cell_start;
  c.inv_id = inv_id;
  c.fx = fx;
  c.fy = fy;
  c.fz = fz;
  c.counters = cnt.c;
  c.n = n;
  c.i0 = 0;
  c.i1 = n;
  c.gxq = gb ? gb->xq : nullptr;
  c.gid = gb ? gb->id : nullptr;
  c.gcell_start = gb ? gb->cell_start : nullptr;
  if (gb) launch_prec<true>(prec, c, nq, part, st);
  else launch_prec<false>(prec, c, nq, part, st);
}

}  // namespace rbe
