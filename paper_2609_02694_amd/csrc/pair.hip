// Near-field force (Sec. 2.1, Eq. 7-8, 10-11): erfc-screened Coulomb plus
// 12-6 Lennard-Jones over a cell list, with the core-shell random batch list.
//
// Full neighbour sums per particle i (cell order), no atomics. Two forms:
// plain sums run one thread per particle, each walking the stencil rows of
// its own cell; the random batch list runs one wave per cluster of 8
// consecutive particles: lane l takes i = cluster[l / 8] and every 8th record
// of one candidate sequence shared by the wave (the union of the cluster's
// stencils), so the candidate loads are contiguous and the loop is uniform
// (pair_device.h, cluster traversal); the 8 partial sums of an i are added
// in a fixed order at the end.
//
// Species blocks: charged particles occupy keys [0, C), neutral ones
// [C, 2C). Coulomb terms only involve charged pairs, so without the random
// batch list a charged i walks the charged block out to r_coul and the
// neutral block out to r_lj; a neutral i walks both blocks out to r_lj.
//
// Random batch list (Eq. 10-11): every j within r_coul is classified with the
// squared distance computed without contraction (the same IEEE expression as
// the CPU oracle). Core terms (r^2 <= r_core^2) are summed exactly. Shell
// members (r_core^2 < r^2 <= r_coul^2) are counted, #S_i, and ranked by the
// 32-bit key of Eq. 11's batch: the batch B_i is the min(p, #S_i) members
// with the smallest keys, summed with the weight #S_i/|B_i|. Selection in one
// pass: keys below a threshold T are appended to the cluster's LDS buffer.
// T is chosen so that about 3p keys fall below it for the mean shell size; if
// the buffer ends with fewer than min(p, #S_i) keys or overflows, a pass that
// only collects keys is repeated with T moved by bisection (keys are distinct,
// so some T always works). The batch is read back through the key's inverse
// (key -> id_j -> sorted slot) and its terms use the minimum image.
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
  const int32_t *__restrict__ nq_ptr;         // charged count (device): [0, nq) charged, [nq, n) neutral
  int charged;                                // this launch: 1 the charged range, 0 the neutral range
  int64_t n;                                  // all particles
  // ghost shell (GHOST kernels only)
  const double4 *__restrict__ gxq;
  const int32_t *__restrict__ gid;
  const int32_t *__restrict__ gcell_start;
};

// Cluster walk of one species block for a row group.
template <bool GHOST, bool WITH_ID, class Fn>
__device__ inline void walk(const PairCtx &c, int blk, int xa, int xb, int cy, int cz, const Sten &s, int b,
                            Fn &&fn) {
  auto no_tick = []() {};
  if (GHOST)
    cluster_walk_ghost<WITH_ID>(c.pp.g, c.cell_start, c.xq, c.ids, c.gcell_start, c.gxq, c.gid, (int)c.n, blk, xa, xb,
                                cy, cz, s, b, fn, no_tick);
  else
    cluster_walk<WITH_ID>(c.pp.g, c.cell_start, c.xq, c.ids, (int64_t)blk * c.pp.g.ncell, xa, xb, cy, cz, s, b, fn,
                          no_tick);
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

// Particle range of this launch, read on the device (the charged count is the
// first neutral cell start), and the first particle of this block's share of
// per_block particles: the grid is sized for all n particles, blocks past the
// range's share exit at once, and the active blocks are spread over the XCDs
// (each XCD takes a contiguous run of the range).
__device__ inline bool part_block(const PairCtx &c, int per_block, int64_t *first, int64_t *end) {
  const int64_t nq = *c.nq_ptr;
  const int64_t a = c.charged ? 0 : nq, b = c.charged ? nq : c.n;
  const int64_t nb = (b - a + per_block - 1) / per_block;
  if ((int64_t)blockIdx.x >= nb) return false;
  *first = a + xcd_block(blockIdx.x, nb) * per_block;
  *end = b;
  return true;
}

// i-side data of a cluster lane.
struct ClusterI {
  int a, b;
  bool valid;
  int64_t i;
  double xi, yi, zi, qi;
  int cx, cy, cz;
};

__device__ inline ClusterI load_cluster_i(const PairCtx &c, int64_t first, int64_t end) {
  ClusterI r;
  const int lane = threadIdx.x;
  r.a = lane / kCJ;
  r.b = lane % kCJ;
  const int64_t i_raw = first + r.a;
  r.valid = i_raw < end;
  r.i = r.valid ? i_raw : end - 1;
  const double4 p = c.xq[r.i];
  r.xi = p.x;
  r.yi = p.y;
  r.zi = p.z;
  r.qi = p.w;
  const Grid &g = c.pp.g;
  r.cx = cell_coord(p.x, g.inv_h[0], g.nx);
  r.cy = cell_coord(p.y, g.inv_h[1], g.ny);
  r.cz = cell_coord(p.z, g.inv_h[2], g.nz);
  return r;
}

// Periodic or ghost-shell stencil walk of one particle (thread form).
template <bool GHOST, bool WITH_ID, class Fn, class RowEnd>
__device__ inline void stencil(const PairCtx &c, int blk, int cx, int cy, int cz, const Sten &s, const Reach &R,
                               Fn &&fn, RowEnd &&row_end) {
  if (GHOST)
    for_stencil_ghost<WITH_ID>(c.pp.g, c.cell_start, c.xq, c.ids, c.gcell_start, c.gxq, c.gid, (int)c.n, blk, cx, cy,
                               cz, s, R, fn, row_end);
  else
    for_stencil<WITH_ID>(c.pp.g, c.cell_start, c.xq, c.ids, blk, cx, cy, cz, s, R, fn, 0, row_end);
}

// Plain cutoff sums, one thread per particle i walking its own stencil (on
// MI355X this beats the cluster form when most candidates within reach are
// summed, i.e. without the shell test of the random batch list). MODE 0:
// neutral i (LJ over both species blocks out to r_lj); MODE 1: charged i
// (charged block out to max(r_coul, r_lj), neutral block out to r_lj); MODE
// 2: charged i, screened Coulomb terms only (charged block out to r_coul),
// added to f, which holds the LJ terms of the tile pass.
// Occupancy asked of the compiler: FP32 forms five (charged) or six
// (neutral) waves per SIMD, the most without spills once a row's partial
// sums are held; FP64 forms three or seven (measured best; the FP64 charged
// form spills at four).
template <bool F32, bool COUNT, int MODE, bool GHOST>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(F32 ? (MODE ? 5 : 6) : (MODE ? 3 : 7))))
k_pair_plain(PairCtx c) {
  static_assert(MODE >= 0 && MODE <= 2, "mode");
  int64_t first, end;
  if (!part_block(c, blockDim.x, &first, &end)) return;
  const int64_t i = first + threadIdx.x;
  if (i >= end) return;
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
    if (j == (int)i) return;  // ghosts are indexed from n on
    if (r2 <= pp.rq2) {
      acc.template add_row<true>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
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
    if (j == (int)i) return;  // ghosts are indexed from n on
    if (r2 <= pp.rlj2) {
      acc.template add_row<false>(pp, c.pf, r2, qi, pj.w, dx, dy, dz);
      if (COUNT) n_lj += pp.do_lj;
    }
  };
  auto row_end = [&]() { acc.flush_row(); };
  const Reach rq{xi, yi, zi, pp.rq2}, rlj{xi, yi, zi, pp.rlj2};
  if (MODE == 2) {
    // pp.do_lj is off for this launch: visit_q adds the screened Coulomb term only
    const Reach rc{xi, yi, zi, pp.rc2};
    stencil<GHOST, false>(c, 0, cx, cy, cz, pp.s_coul, rc, visit_q, row_end);
    c.fx[i] += acc.get(0);
    c.fy[i] += acc.get(1);
    c.fz[i] += acc.get(2);
  } else {
    if (MODE == 1) {
      stencil<GHOST, false>(c, 0, cx, cy, cz, pp.s_coul, rq, visit_q, row_end);
      if (pp.do_lj) stencil<GHOST, false>(c, 1, cx, cy, cz, pp.s_lj, rlj, visit_lj, row_end);
    } else if (pp.do_lj) {
      stencil<GHOST, false>(c, 0, cx, cy, cz, pp.s_lj, rlj, visit_lj, row_end);
      stencil<GHOST, false>(c, 1, cx, cy, cz, pp.s_lj, rlj, visit_lj, row_end);
    }
    c.fx[i] = acc.get(0);
    c.fy[i] = acc.get(1);
    c.fz[i] = acc.get(2);
  }
  flush_counts<COUNT>(c, n_coul, n_lj, n_tested, 0);
}

// Random batch list (Eq. 10-11) for the particles of the launch range: exact
// core, counted and ranked shell, one walk of both species blocks out to
// r_coul.
// QSHELL: the shell holds charged particles only (variant of Eq. 10; the
// neutral j beyond the core then carry no force, since r_lj <= r_core).
template <bool F32, bool COUNT, bool GHOST, bool QSHELL>
__global__ void __launch_bounds__(64, 5) k_pair_rbl(PairCtx c) {
  __shared__ uint32_t kbuf[kCI * kShellCap];
  __shared__ uint32_t ksel[kCI * RBE_MAX_SHELL_BATCH];
  __shared__ int kcnt[kCI];
  int64_t first, end;
  if (!part_block(c, kCI, &first, &end)) return;
  const ClusterI I = load_cluster_i(c, first, end);
  const PairParams &pp = c.pp;
  const Grid &g = pp.g;
  const int p = pp.p_shell;
  const ShellKey sk = shell_key_of(pp.shell_key, c.ids[I.i]);
  ForceAcc<F32> acc;
  unsigned long long n_coul = 0, n_lj = 0, n_tested = 0;
  int ns = 0;  // shell members seen by this lane
  // keys below T are collected; the mean shell of the charged-only variant
  // holds charged particles, whose count is known on the device only
  uint64_t T = QSHELL ? shell_first_threshold(pp, *c.nq_ptr) : pp.shell_T0;
  bool in_group = false;
  if (I.b == 0) kcnt[I.a] = 0;
  __syncthreads();
  auto collect = [&](uint32_t k) {
    if ((uint64_t)k < T) {
      const int s = atomicAdd(&kcnt[I.a], 1);
      if (s < kShellCap) kbuf[I.a * kShellCap + s] = k;
    }
  };
  auto visit = [&](bool ok, int j, const double4 &pj, int idj, double shx, double shy, double shz) {
    const double dx = (I.xi - pj.x) - shx, dy = (I.yi - pj.y) - shy, dz = (I.zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    // flat predicates (bitwise, so no branch per condition)
    // j indexes natives, or ghosts offset by n: only i itself has j == i (its
    // periodic images lie at least L >= 2 r_coul away)
    const bool live = ok & in_group & (j != (int)I.i);
    const bool core = live & (r2 <= pp.rcore2);
    const bool shell = live & (r2 > pp.rcore2) & (r2 <= pp.rc2) & (!QSHELL | (pj.w != 0.0));
    if (COUNT) n_tested += ok & in_group;
    if (core) {
      acc.template add<true, true>(pp, c.pf, r2, I.qi, pj.w, dx, dy, dz);
      if (COUNT) {
        n_coul += (pp.do_coul && I.qi != 0.0 && pj.w != 0.0);
        n_lj += (pp.do_lj && r2 <= pp.rlj2);
      }
    }
    ns += shell;
    if (shell) collect(shell_rank(sk, idj));
  };
  auto visit_collect = [&](bool ok, int, const double4 &pj, int idj, double shx, double shy, double shz) {
    const double dx = (I.xi - pj.x) - shx, dy = (I.yi - pj.y) - shy, dz = (I.zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (ok & in_group & (r2 > pp.rcore2) & (r2 <= pp.rc2) & (!QSHELL | (pj.w != 0.0)))
      collect(shell_rank(sk, idj));
  };
  const int64_t rowkey = (int64_t)I.cz * g.ny + I.cy;
  auto walk_all = [&](bool active, auto &&fn) {
    for_each_row_group(active, rowkey, I.cx, [&](bool in, int leader, int xa, int xb) {
      in_group = in;
      const int cy = __shfl(I.cy, leader, 64), cz = __shfl(I.cz, leader, 64);
      walk<GHOST, true>(c, 0, xa, xb, cy, cz, pp.s_coul, I.b, fn);
      // with a charged-only shell the neutral block matters inside the core
      // only (r_lj <= r_core): its walk covers r_core instead of r_coul
      walk<GHOST, true>(c, 1, xa, xb, cy, cz, QSHELL ? pp.s_core : pp.s_coul, I.b, fn);
    });
  };
  walk_all(I.valid, visit);
  __syncthreads();
  const int m = sum_j_lanes(ns);  // #S_i
  const int need = m < p ? m : p;
  int got = kcnt[I.a];
  // bisection on T when the buffer missed [need, cap] (rare; distinct keys
  // end it within 33 rounds, the bound only guards against duplicate ids,
  // which the inverse id map reports)
  uint64_t lo = 0, hi = 1ull << 32;
  bool pend = I.valid && need > 0 && (got < need || got > kShellCap);
  for (int round = 0; __any(pend) && round < 40; ++round) {
    if (pend) {
      if (got < need) lo = T;
      else hi = T;
      T = (m <= kShellCap) ? (1ull << 32) : lo + (hi - lo) / 2;
    }
    __syncthreads();
    if (pend && I.b == 0) kcnt[I.a] = 0;
    __syncthreads();
    walk_all(pend, visit_collect);
    __syncthreads();
    if (pend) got = kcnt[I.a];
    pend = pend && (got < need || got > kShellCap);
  }
  got = min(got, kShellCap);
  const int nb = min(need, got);  // = need unless ids repeat
  // ranks of the collected keys (distinct); the first `need` form the batch
  if (I.valid && nb > 0) {
    const uint32_t *kb = kbuf + I.a * kShellCap;
    for (int t = I.b; t < got; t += kCJ) {
      const uint32_t k = kb[t];
      int rank = 0;
      for (int u = 0; u < got; ++u) rank += kb[u] < k;
      if (rank < nb) ksel[I.a * RBE_MAX_SHELL_BATCH + rank] = k;
    }
  }
  __syncthreads();
  ForceAcc<F32> sh;
  if (I.valid) {
    for (int r = I.b; r < nb; r += kCJ) {
      const int32_t idj = shell_id_of(sk, ksel[I.a * RBE_MAX_SHELL_BATCH + r]);
      if ((uint32_t)idj >= (uint32_t)c.n) continue;  // bad ids (flagged by the inverse map)
      const int j = c.inv_id[idj];
      if ((uint32_t)j >= (uint32_t)c.n) continue;
      const double4 pj = c.xq[j];
      const double dx = min_image(I.xi - pj.x, g.L[0]);
      const double dy = min_image(I.yi - pj.y, g.L[1]);
      const double dz = min_image(I.zi - pj.z, g.L[2]);
      const double r2 = sq_dist(dx, dy, dz);
      sh.template add<true, true>(pp, c.pf, r2, I.qi, pj.w, dx, dy, dz);
      if (COUNT) {
        n_coul += (pp.do_coul && I.qi != 0.0 && pj.w != 0.0);
        n_lj += (pp.do_lj && r2 <= pp.rlj2);
      }
    }
  }
  double f0 = sum_j_lanes(acc.get(0)), f1 = sum_j_lanes(acc.get(1)), f2 = sum_j_lanes(acc.get(2));
  const double s0 = sum_j_lanes(sh.get(0)), s1 = sum_j_lanes(sh.get(1)), s2 = sum_j_lanes(sh.get(2));
  if (nb > 0) {
    const double scale = (double)m / (double)nb;
    f0 = fma(scale, s0, f0);
    f1 = fma(scale, s1, f1);
    f2 = fma(scale, s2, f2);
  }
  if (I.valid && I.b == 0) {
    c.fx[I.i] = f0;
    c.fy[I.i] = f1;
    c.fz[I.i] = f2;
  }
  flush_counts<COUNT>(c, n_coul, n_lj, n_tested, I.b == 0 && I.valid ? (unsigned long long)m : 0ull);
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

// Thread form: 256 particles per block. Cluster form: one wave of kCI
// particles per block. Grids cover all n particles (the part's range is read
// on the device; surplus blocks exit at once).
template <class K>
static void launch_threads(K kernel, PairCtx c, hipStream_t st) {
  kernel<<<(unsigned)((c.n + 255) / 256), 256, 0, st>>>(c);
}
template <class K>
static void launch_clusters(K kernel, PairCtx c, hipStream_t st) {
  kernel<<<(unsigned)((c.n + kCI - 1) / kCI), 64, 0, st>>>(c);
}

// Charged particles occupy [0, nq) of the sorted order, neutral ones [nq, n).
// With the random batch list the charged particles take the RBL kernel; the
// neutral ones too when r_lj > r_core (their LJ terms then reach the shell),
// else their sums are plain (every LJ term lies in the core).
// part: PAIR_PART_CHARGED, PAIR_PART_SHELL (nothing left to do: the shell is
// fused into the charged part) or PAIR_PART_NEUTRAL.
template <bool F32, bool COUNT, bool GHOST>
static void launch_part(PairCtx c, int part, hipStream_t st) {
  const PairParams pp = c.pp;
  if (part == PAIR_PART_CHARGED) {
    c.charged = 1;
    if (pp.rbl && pp.shell_charged) launch_clusters(k_pair_rbl<F32, COUNT, GHOST, true>, c, st);
    else if (pp.rbl) launch_clusters(k_pair_rbl<F32, COUNT, GHOST, false>, c, st);
    else launch_threads(k_pair_plain<F32, COUNT, 1, GHOST>, c, st);
  } else if (part == PAIR_PART_COULOMB) {
    c.charged = 1;
    c.pp.do_lj = 0;
    launch_threads(k_pair_plain<F32, COUNT, 2, GHOST>, c, st);
  } else if (part == PAIR_PART_NEUTRAL) {
    c.charged = 0;
    if (pp.rbl && pp.rlj2 > pp.rcore2 && pp.do_lj) launch_clusters(k_pair_rbl<F32, COUNT, GHOST, false>, c, st);
    else launch_threads(k_pair_plain<F32, COUNT, 0, GHOST>, c, st);
  }
}

template <bool GHOST>
static void launch_prec(int prec, PairCtx c, int part, hipStream_t st) {
  if (prec == RBE_FP32C) {
    if (c.counters) launch_part<true, true, GHOST>(c, part, st);
    else launch_part<true, false, GHOST>(c, part, st);
  } else {
    if (c.counters) launch_part<false, true, GHOST>(c, part, st);
    else launch_part<false, false, GHOST>(c, part, st);
  }
}

void launch_pair(int prec, int part, const PairParams &pp, int64_t n, const int32_t *nq, const Sorted &s,
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
  c.nq_ptr = nq;
  c.charged = part == PAIR_PART_CHARGED;
  c.gxq = gb ? gb->xq : nullptr;
  c.gid = gb ? gb->id : nullptr;
  c.gcell_start = gb ? gb->cell_start : nullptr;
  if (gb) launch_prec<true>(prec, c, part, st);
  else launch_prec<false>(prec, c, part, st);
}

}  // namespace rbe
