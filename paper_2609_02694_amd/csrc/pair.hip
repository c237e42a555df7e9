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
#include "pair_device.h"

namespace rbe {

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

PairF32 make_pair_f32(const PairParams &pp) {
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
  c.pf = make_pair_f32(pp);
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
