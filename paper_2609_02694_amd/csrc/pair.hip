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

__device__ inline double pair_scalar_f64(const PairParams &pp, double r2, double qi, double qj) {
  double f = 0.0;
  if (pp.do_coul && r2 <= pp.rc2 && qi != 0.0 && qj != 0.0) {
    const double r = sqrt(r2);
    const double G = erfc(pp.sqrt_alpha * r) / (r2 * r) + pp.two_sqrt_alpha_over_sqrt_pi * exp(-pp.alpha * r2) / r2;
    f += pp.kc * qi * qj * G;
  }
  if (pp.do_lj && r2 <= pp.rlj2) {
    const double s2 = pp.sig2 / r2;
    const double s6 = s2 * s2 * s2;
    f += pp.eps24 * (2.0 * s6 * s6 - s6) / r2;
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

// Calls fn(j, shx, shy, shz) for every particle j of species block `blk` in
// the (2s+1)^3 cells around (cx, cy, cz); (shx, shy, shz) is the image shift
// of j (its image lies at r_j + shift).
template <class Fn>
__device__ inline void for_stencil(const Grid &g, const int32_t *__restrict__ cell_start, int blk, int cx, int cy,
                                   int cz, int s, Fn &&fn) {
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
        const double shx = (double)qx * g.L[0];
        for (int j = j0; j < j1; ++j) fn(j, shx, shy, shz);
        a = b + 1;
      }
    }
  }
}

constexpr int kShellCap = RBE_MAX_SHELL_BATCH;

// Accumulator of the per-particle force in the two precision forms.
template <bool F32>
struct ForceAcc;
template <>
struct ForceAcc<false> {
  double v[3] = {0.0, 0.0, 0.0};
  __device__ inline void add(const PairParams &pp, const PairF32 &, double r2, double qi, double qj, double dx,
                             double dy, double dz) {
    const double sc = pair_scalar_f64(pp, r2, qi, qj);
    v[0] = fma(sc, dx, v[0]);
    v[1] = fma(sc, dy, v[1]);
    v[2] = fma(sc, dz, v[2]);
  }
  __device__ inline double get(int k) const { return v[k]; }
};
template <>
struct ForceAcc<true> {
  Kahan3 k;
  __device__ inline void add(const PairParams &pp, const PairF32 &pf, double r2, double qi, double qj, double dx,
                             double dy, double dz) {
    const float sc = pair_scalar_f32(pp, pf, r2, (float)(qi * qj));
    k.add(0, sc * (float)dx);
    k.add(1, sc * (float)dy);
    k.add(2, sc * (float)dz);
  }
  __device__ inline double get(int c) const { return k.get(c); }
};

template <bool F32, bool COUNT>
__global__ void __launch_bounds__(256) k_pair(PairParams pp, PairF32 pf, int64_t n, const double4 *__restrict__ xq,
                                              const int32_t *__restrict__ ids,
                                              const int32_t *__restrict__ cell_start,
                                              const int32_t *__restrict__ inv_id, double *__restrict__ fx,
                                              double *__restrict__ fy, double *__restrict__ fz,
                                              unsigned long long *__restrict__ counters) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Grid &g = pp.g;
  const double4 pi4 = xq[i];
  const double xi = pi4.x, yi = pi4.y, zi = pi4.z, qi = pi4.w;
  const int cx = cell_coord(xi, g.inv_h[0], g.nx);
  const int cy = cell_coord(yi, g.inv_h[1], g.ny);
  const int cz = cell_coord(zi, g.inv_h[2], g.nz);
  ForceAcc<F32> acc;
  unsigned long long n_coul = 0, n_lj = 0, n_tested = 0, n_shell = 0;
  const bool charged = qi != 0.0;
  const bool shell_on = pp.rbl && (charged || pp.rlj2 > pp.rcore2);
  auto count_pair = [&](double r2, double qj) {
    if (COUNT) {
      n_coul += (pp.do_coul && r2 <= pp.rc2 && charged && qj != 0.0);
      n_lj += (pp.do_lj && r2 <= pp.rlj2);
    }
  };

  if (!shell_on) {
    // plain cutoff sums
    auto plain = [&](int j, double shx, double shy, double shz) {
      const double4 pj = xq[j];
      const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
      const double r2 = sq_dist(dx, dy, dz);
      if (COUNT) ++n_tested;
      if (r2 == 0.0 && j == (int)i) return;
      if (r2 <= pp.rc2 || r2 <= pp.rlj2) {
        acc.add(pp, pf, r2, qi, pj.w, dx, dy, dz);
        count_pair(r2, pj.w);
      }
    };
    if (charged) {
      for_stencil(g, cell_start, 0, cx, cy, cz, pp.s_coul, plain);
      if (pp.do_lj) for_stencil(g, cell_start, 1, cx, cy, cz, pp.s_lj, plain);
    } else if (pp.do_lj) {
      for_stencil(g, cell_start, 0, cx, cy, cz, pp.s_lj, plain);
      for_stencil(g, cell_start, 1, cx, cy, cz, pp.s_lj, plain);
    }
  } else {
    // random batch list: exact core, ranked shell
    uint32_t keys[kShellCap];
#pragma unroll
    for (int t = 0; t < kShellCap; ++t) keys[t] = 0xFFFFFFFFu;
    const ShellKey sk = shell_key_of(pp.shell_key, ids[i]);
    int ns = 0;
    auto rbl = [&](int j, double shx, double shy, double shz) {
      const double4 pj = xq[j];
      const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
      const double r2 = sq_dist(dx, dy, dz);
      if (COUNT) ++n_tested;
      if (r2 == 0.0 && j == (int)i) return;
      if (r2 <= pp.rcore2) {
        acc.add(pp, pf, r2, qi, pj.w, dx, dy, dz);
        count_pair(r2, pj.w);
      } else if (r2 <= pp.rc2) {
        ++ns;
        const uint32_t k = shell_rank(sk, ids[j]);
        if (k < keys[kShellCap - 1]) {
          uint32_t carry = k;
#pragma unroll
          for (int t = 0; t < kShellCap; ++t) {
            const uint32_t lo = min(keys[t], carry);
            carry = max(keys[t], carry);
            keys[t] = lo;
          }
        }
      }
    };
    for_stencil(g, cell_start, 0, cx, cy, cz, pp.s_coul, rbl);
    for_stencil(g, cell_start, 1, cx, cy, cz, pp.s_coul, rbl);
    if (ns > 0) {
      const int nb = ns < pp.p_shell ? ns : pp.p_shell;
      ForceAcc<F32> sh;
#pragma unroll
      for (int t = 0; t < kShellCap; ++t) {
        if (t < nb) {
          const int32_t idj = shell_id_of(sk, keys[t]);
          if ((uint32_t)idj >= (uint32_t)n) continue;  // bad ids (flagged by the inverse map)
          const int j = inv_id[idj];
          if ((uint32_t)j >= (uint32_t)n) continue;
          const double4 pj = xq[j];
          const double dx = min_image(xi - pj.x, g.L[0]);
          const double dy = min_image(yi - pj.y, g.L[1]);
          const double dz = min_image(zi - pj.z, g.L[2]);
          const double r2 = sq_dist(dx, dy, dz);
          sh.add(pp, pf, r2, qi, pj.w, dx, dy, dz);
          count_pair(r2, pj.w);
        }
      }
      const double scale = (double)ns / (double)nb;
      fx[i] = fma(scale, sh.get(0), acc.get(0));
      fy[i] = fma(scale, sh.get(1), acc.get(1));
      fz[i] = fma(scale, sh.get(2), acc.get(2));
    } else {
      fx[i] = acc.get(0);
      fy[i] = acc.get(1);
      fz[i] = acc.get(2);
    }
    if (COUNT) n_shell = (unsigned long long)ns;
  }
  if (!shell_on) {
    fx[i] = acc.get(0);
    fy[i] = acc.get(1);
    fz[i] = acc.get(2);
  }
  if (COUNT) {
    atomicAdd(&counters[0], n_coul);
    atomicAdd(&counters[1], n_lj);
    atomicAdd(&counters[2], n_tested);
    atomicAdd(&counters[3], n_shell);
  }
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

template <bool F32>
static void launch_pair(const PairParams &pp, int64_t n, const Sorted &s, const int32_t *cell_start,
                        const int32_t *inv_id, double *fx, double *fy, double *fz, PairCounters cnt, hipStream_t st) {
  if (n <= 0) return;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  const PairF32 pf = make_f32(pp);
  if (cnt.c)
    k_pair<F32, true><<<blocks, 256, 0, st>>>(pp, pf, n, s.xq, s.id, cell_start, inv_id, fx, fy, fz, cnt.c);
  else
    k_pair<F32, false><<<blocks, 256, 0, st>>>(pp, pf, n, s.xq, s.id, cell_start, inv_id, fx, fy, fz, nullptr);
}

void launch_pair_f64(const PairParams &pp, int64_t n, const Sorted &s, const int32_t *cell_start,
                     const int32_t *inv_id, double *fx, double *fy, double *fz, PairCounters cnt, hipStream_t st) {
  launch_pair<false>(pp, n, s, cell_start, inv_id, fx, fy, fz, cnt, st);
}

void launch_pair_f32c(const PairParams &pp, int64_t n, const Sorted &s, const int32_t *cell_start,
                      const int32_t *inv_id, double *fx, double *fy, double *fz, PairCounters cnt, hipStream_t st) {
  launch_pair<true>(pp, n, s, cell_start, inv_id, fx, fy, fz, cnt, st);
}

}  // namespace rbe
