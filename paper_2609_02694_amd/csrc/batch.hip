// Batched form: many independent systems ("replicas") of uneven size advanced
// together, three launches per velocity-Verlet step.
//
// All replicas live in concatenated arrays; replica r owns particles
// [p0, p0 + n) and binning keys [c0, c0 + 2 C_r) (its charged cells, then its
// neutral cells). A persistent kernel runs the step for every replica, phase
// by phase, with a grid-wide barrier between phases, in two launches: P0-P6,
// then P7-P9. Between them a plain kernel sums the near field of every
// particle, with the occupancy of its own register count:
//
//   P0  half-kick + drift + wrap; binning keys + histogram; mode sample of
//       every replica (Eq. 9)
//   P1  scan: tile sums of the concatenated histogram
//   P2  scan: one block scans the tile sums
//   P3  scan: cell starts (one exclusive scan serves every replica, because
//       replica r's keys and particles both follow those of replicas < r)
//   P4  provisional scatter (atomic slots)
//   P5  stable placement (each bucket's entries in increasing input order)
//   P6  reorder of the state and packing of the sorted records
//   --  near field of every particle (k_batch_near)
//   P7  structure-factor partials (chunk x mode)
//   P8  structure factors: fixed-order sum of the chunk partials per mode
//   P9  Fourier gather + second half-kick
//
// The grid is sized to the kernel's resident capacity, so every block is
// resident and the barrier cannot wait on a block that never starts; the
// barrier's wait is still bounded in time and reports an error instead of
// hanging. Data written inside the kernel is read only through vector loads
// after an agent-scope fence.
#include "fourier_device.h"
#include "pair_device.h"
#include "sampler_device.h"

namespace rbe {

constexpr int kBatchThreads = 256;
constexpr int kScanTileB = kBatchThreads * 8;
constexpr uint64_t kBarrierTimeoutTicks = 200000000ull;  // 2 s at the 100 MHz wall clock

// Grid-wide barrier. A wait longer than the time limit flags kErrBarrier;
// once that flag is up no block waits again, so a launch whose blocks were
// not all resident still ends (with its result reported as failed).
// Every wave waits until its own stores have reached the L2 (s_waitcnt 0)
// before the block barrier; one wave per block then releases the block's
// stores at agent scope with its arrival (the L2 write-back covers them all)
// and, after the wait, acquires the other blocks' (invalidating the caches
// every wave of the block reads through). Fences in every wave would repeat
// the write-back and the invalidation per wave.
__device__ inline void grid_barrier(unsigned *bar, int *err) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    // the arrival releases the block's stores (and acquires the earlier
    // arrivals' for the last one); the generation read before it needs no
    // ordering of its own
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
    if (arrived == gridDim.x) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      const uint64_t t0 = wall_clock64();
      // relaxed polls (an acquire would invalidate the caches on every poll);
      // the fence after the wait acquires
      while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        if (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kErrBarrier) break;
        __builtin_amdgcn_s_sleep(4);
        if (wall_clock64() - t0 > kBarrierTimeoutTicks) {
          atomicOr(err, kErrBarrier);
          break;
        }
      }
    }
    __threadfence();
  }
  __syncthreads();
}

__device__ inline int block_scan_excl(int v, int *lds, int *total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) lds[wave] = incl;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < kBatchThreads / 64; ++w) {
    const int s = lds[w];
    if (w < wave) off += s;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + incl - v;
}

// Plain near-field sums of one particle (no random batch list, no ghosts),
// one thread walking the stencil rows of its own cell in its replica.
template <bool F32>
__device__ inline void batch_pair(const BatchArgs &a, const RepDesc &R, int64_t i) {
  const Grid &g = R.g;
  const PairParams &pp = a.pp;
  const double4 pi4 = a.xq[i];
  const double xi = pi4.x, yi = pi4.y, zi = pi4.z, qi = pi4.w;
  const int cx = cell_coord(xi, g.inv_h[0], g.nx);
  const int cy = cell_coord(yi, g.inv_h[1], g.ny);
  const int cz = cell_coord(zi, g.inv_h[2], g.nz);
  ForceAcc<F32> acc;
  auto visit_q = [&](int j, const double4 &pj, int, double shx, double shy, double shz) {
    const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (r2 == 0.0 && j == (int)i) return;
    if (r2 <= pp.rq2) acc.template add_row<true>(pp, a.pf, r2, qi, pj.w, dx, dy, dz);
  };
  auto visit_lj = [&](int j, const double4 &pj, int, double shx, double shy, double shz) {
    const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
    const double r2 = sq_dist(dx, dy, dz);
    if (r2 == 0.0 && j == (int)i) return;
    if (r2 <= pp.rlj2) acc.template add_row<false>(pp, a.pf, r2, qi, pj.w, dx, dy, dz);
  };
  // FP32C: a row's terms summed plainly, the row sum added with Kahan compensation
  auto row_end = [&]() { acc.flush_row(); };
  const Reach rq{xi, yi, zi, pp.rq2}, rlj{xi, yi, zi, pp.rlj2};
  if (qi != 0.0) {
    if (pp.do_coul || pp.do_lj)
      for_stencil<false>(g, a.cell_start, a.xq, a.sid, 0, cx, cy, cz, R.s_coul, rq, visit_q, R.c0, row_end);
    if (pp.do_lj)
      for_stencil<false>(g, a.cell_start, a.xq, a.sid, 1, cx, cy, cz, R.s_lj, rlj, visit_lj, R.c0, row_end);
  } else if (pp.do_lj) {
    for_stencil<false>(g, a.cell_start, a.xq, a.sid, 0, cx, cy, cz, R.s_lj, rlj, visit_lj, R.c0, row_end);
    for_stencil<false>(g, a.cell_start, a.xq, a.sid, 1, cx, cy, cz, R.s_lj, rlj, visit_lj, R.c0, row_end);
  }
  a.ofx[i] = acc.get(0);
  a.ofy[i] = acc.get(1);
  a.ofz[i] = acc.get(2);
}


template <bool F32>
__global__ void __launch_bounds__(kBatchThreads) k_batch_step(BatchArgs a) {
  __shared__ int lds[kBatchThreads / 64];
  const int tid = threadIdx.x;
  const int64_t gtid = xcd_block(blockIdx.x, gridDim.x) * kBatchThreads + tid;
  const int64_t gstride = (int64_t)gridDim.x * kBatchThreads;
  const int lane = tid & 63;
  const int64_t gwave = xcd_block(blockIdx.x, gridDim.x) * (kBatchThreads / 64) + (tid >> 6);
  const int64_t nwaves = (int64_t)gridDim.x * (kBatchThreads / 64);
  const int P = a.P;
  const bool do_far = a.do_far != 0;
  const uint64_t eval = *((volatile uint64_t *)a.eval);

  if (a.launch_part == 1) {
    // ---- P0: drift, keys + histogram, mode sample ----------------------------
    // wave-uniform trip count (every lane takes part in the slot vote)
    for (int64_t i = gtid; i - lane < a.ntot; i += gstride) {
      const bool active = i < a.ntot;
      int k = -1 - lane;  // lanes past the end: a key no other lane has
      if (active) {
        const RepDesc &R = a.reps[a.rep_of[i]];
        double x = a.ix[i], y = a.iy[i], z = a.iz[i];
        if (a.mode == 0) {
          const double u = a.ivx[i] + a.h * a.ifx[i], v = a.ivy[i] + a.h * a.ify[i], w = a.ivz[i] + a.h * a.ifz[i];
          a.ivx[i] = u;
          a.ivy[i] = v;
          a.ivz[i] = w;
          x = wrap_coord(x + a.dt * u, R.g.L[0]);
          y = wrap_coord(y + a.dt * v, R.g.L[1]);
          z = wrap_coord(z + a.dt * w, R.g.L[2]);
          a.ix[i] = x;
          a.iy[i] = y;
          a.iz[i] = z;
          if (!isfinite(u) || !isfinite(v) || !isfinite(w)) atomicOr(a.err, kErrNonFinite);
        } else {
          x = wrap_coord(x, R.g.L[0]);
          y = wrap_coord(y, R.g.L[1]);
          z = wrap_coord(z, R.g.L[2]);
        }
        const int cx = cell_coord(x, R.g.inv_h[0], R.g.nx);
        const int cy = cell_coord(y, R.g.inv_h[1], R.g.ny);
        const int cz = cell_coord(z, R.g.inv_h[2], R.g.nz);
        k = (int)(R.c0 + (a.iq[i] == 0.0 ? R.g.ncell : 0) + (cz * R.g.ny + cy) * R.g.nx + cx);
        a.key[i] = k;
      }
      const int sl = run_slot(k, active, a.count);
      if (active) a.slot[i] = sl;
    }
    if (P > 0) {
      for (int64_t it = gtid; it < (int64_t)a.nrep * P; it += gstride) {
        const int r = (int)(it / P), l = (int)(it % P);
        const RepDesc &R = a.reps[r];
        const uint64_t ek = stream_out(R.seed ^ kTagModes, eval);
        int mv[3];
        if (!draw_mode(R.mt, a.cdf + R.cdf_off, ek, l, mv)) {
          atomicOr(a.err, kErrSampler);
          mv[0] = 1;
          mv[1] = 0;
          mv[2] = 0;
        }
        GatherMode gm;
        gm.mx = (double)mv[0];
        gm.my = (double)mv[1];
        gm.mz = (double)mv[2];
        gm.a = 0.0;
        gm.b = 0.0;
        gather_floats(gm);
        a.modes[it] = gm;
        a.wk[it] = mode_weight(R.mt, P, mv[0], mv[1], mv[2]);
      }
    }
    grid_barrier(a.bar, a.err);

    // ---- P1: tile sums -------------------------------------------------------
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
      const int64_t base = (int64_t)t * kScanTileB + (int64_t)tid * 8;
      int s = 0;
      for (int k = 0; k < 8; ++k)
        if (base + k < a.nkeys) s += a.count[base + k];
      int tot;
      block_scan_excl(s, lds, &tot);
      if (tid == 0) a.tile_sum[t] = tot;
    }
    grid_barrier(a.bar, a.err);

    // ---- P2: scan of the tile sums (one block) --------------------------------
    if (blockIdx.x == 0) {
      int carry = 0;
      for (int b = 0; b < a.ntiles; b += kBatchThreads) {
        const int t = b + tid;
        const int v = t < a.ntiles ? a.tile_sum[t] : 0;
        int tot;
        const int ex = block_scan_excl(v, lds, &tot);
        if (t < a.ntiles) a.tile_sum[t] = carry + ex;
        carry += tot;
      }
      if (tid == 0) a.cell_start[a.nkeys] = carry;
    }
    grid_barrier(a.bar, a.err);

    // ---- P3: cell starts -------------------------------------------------------
    for (int t = blockIdx.x; t < a.ntiles; t += gridDim.x) {
      const int64_t base = (int64_t)t * kScanTileB + (int64_t)tid * 8;
      int v[8];
      int s = 0;
      for (int k = 0; k < 8; ++k) {
        v[k] = base + k < a.nkeys ? a.count[base + k] : 0;
        s += v[k];
      }
      int tot;
      int run = a.tile_sum[t] + block_scan_excl(s, lds, &tot);
      for (int k = 0; k < 8; ++k) {
        if (base + k < a.nkeys) a.cell_start[base + k] = run;
        run += v[k];
      }
    }
    grid_barrier(a.bar, a.err);

    // ---- P4: provisional scatter -----------------------------------------------
    for (int64_t i = gtid; i < a.ntot; i += gstride) a.tmp[a.cell_start[a.key[i]] + a.slot[i]] = (int32_t)i;
    grid_barrier(a.bar, a.err);

    // ---- P5: stable placement; clear the histogram for the next step -----------
    for (int64_t k = gtid; k < a.nkeys; k += gstride) place_bucket(a.cell_start[k], a.cell_start[k + 1], a.tmp, a.perm);
    for (int64_t k = gtid; k < a.nkeys; k += gstride) a.count[k] = 0;
    grid_barrier(a.bar, a.err);

    // ---- P6: reorder + pack ------------------------------------------------------
    for (int64_t k = gtid; k < a.ntot; k += gstride) {
      const int j = a.perm[k];
      const RepDesc &R = a.reps[a.rep_of[k]];
      const double x = wrap_coord(a.ix[j], R.g.L[0]), y = wrap_coord(a.iy[j], R.g.L[1]),
                   z = wrap_coord(a.iz[j], R.g.L[2]), q = a.iq[j];
      const int32_t id = a.iid[j];
      a.ox[k] = x;
      a.oy[k] = y;
      a.oz[k] = z;
      a.oq[k] = q;
      a.oid[k] = id;
      if (a.mode == 0) {
        a.ovx[k] = a.ivx[j];
        a.ovy[k] = a.ivy[j];
        a.ovz[k] = a.ivz[j];
      }
      a.xq[k] = make_double4(x, y, z, q);
      if (q != 0.0) a.sq[k] = make_double4(x / R.g.L[0], y / R.g.L[1], z / R.g.L[2], q);
      a.sid[k] = id;
    }
    grid_barrier(a.bar, a.err);
    return;
  }


  // ---- P7: structure-factor partials (the near field ran in k_batch_near) --------
  if (P > 0 && do_far) {
    const int groups = (P + 63) / 64;
    const int64_t rho_items = *a.rho_items;
    for (int64_t it = gwave; it < rho_items; it += nwaves) {
      // replica of this item: last r with rho_item_off <= it
      int lo = 0, hi = a.nrep - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.reps[mid].rho_item_off <= it) lo = mid;
        else hi = mid - 1;
      }
      const RepDesc &R = a.reps[lo];
      const int local = (int)(it - R.rho_item_off);
      const int chunk = local / groups, grp = local % groups;
      const int l = grp * 64 + lane;
      const bool active = l < P;
      const GatherMode gm = a.modes[(int64_t)lo * P + (active ? l : 0)];
      const int64_t j0 = R.p0 + (int64_t)chunk * R.chunk_len;
      const int64_t j1 = min(R.p0 + (int64_t)R.nq, j0 + R.chunk_len);
      double2 out;
      if (F32) {
        float re = 0.f, rc = 0.f, im = 0.f, ic = 0.f;
#pragma unroll 4
        for (int64_t j = j0; j < j1; ++j) {
          const double4 s = a.sq[j];
          const float t = turn_f32(gm.mx, gm.my, gm.mz, s.x, s.y, s.z);
          const float q = (float)s.w;
          kahan_fma(re, rc, q, __builtin_amdgcn_cosf(t));
          kahan_fma(im, ic, q, __builtin_amdgcn_sinf(t));
        }
        out = make_double2((double)re - (double)rc, (double)im - (double)ic);
      } else {
        double re = 0.0, im = 0.0;
#pragma unroll 4
        for (int64_t j = j0; j < j1; ++j) {
          const double4 s = a.sq[j];
          const double t = turn_fraction(gm.mx, gm.my, gm.mz, s.x, s.y, s.z);
          double sn, cs;
          sincos_turn_f64(t, &sn, &cs);
          re = fma(s.w, cs, re);
          im = fma(s.w, sn, im);
        }
        out = make_double2(re, im);
      }
      if (active) a.part[(int64_t)(R.chunk_off + chunk) * P + l] = out;
    }
  }
  grid_barrier(a.bar, a.err);

  // ---- P8: structure factors and gather coefficients --------------------------
  if (P > 0 && do_far) {
    for (int64_t it = gwave; it < (int64_t)a.nrep * P; it += nwaves) {
      const int r = (int)(it / P), l = (int)(it % P);
      const RepDesc &R = a.reps[r];
      double re = 0.0, im = 0.0;
      for (int c = lane; c < R.nchunks; c += 64) {
        const double2 v = a.part[(int64_t)(R.chunk_off + c) * P + l];
        re += v.x;
        im += v.y;
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        re += __shfl_xor(re, o, 64);
        im += __shfl_xor(im, o, 64);
      }
      if (lane == 0) {
        const double w = a.pp.kc * a.wk[it];
        a.modes[it].a = w * im;
        a.modes[it].b = w * re;
        a.modes[it].af = (float)(w * im);
        a.modes[it].bf = (float)(w * re);
      }
    }
  }
  grid_barrier(a.bar, a.err);

  // ---- P9: Fourier gather + second half-kick -----------------------------------
  for (int64_t i = gtid; i < a.ntot; i += gstride) {
    const int r = a.rep_of[i];
    const RepDesc &R = a.reps[r];
    double fx = a.ofx[i], fy = a.ofy[i], fz = a.ofz[i];
    if (P > 0 && do_far && i < R.p0 + R.nq) {
      const double4 s = a.sq[i];
      const GatherMode *md = a.modes + (int64_t)r * P;
      if (F32) {
        float gx = 0.f, gy = 0.f, gz = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll 4
        for (int l = 0; l < P; ++l) {
          const GatherMode gm = md[l];
          const float t = turn_f32(gm.mx, gm.my, gm.mz, s.x, s.y, s.z);
          const float g = fmaf(gm.af, __builtin_amdgcn_cosf(t), -gm.bf * __builtin_amdgcn_sinf(t));
          kahan_fma(gx, ex, g, gm.mxf);
          kahan_fma(gy, ey, g, gm.myf);
          kahan_fma(gz, ez, g, gm.mzf);
        }
        fx -= s.w * (kTwoPi / R.g.L[0]) * ((double)gx - (double)ex);
        fy -= s.w * (kTwoPi / R.g.L[1]) * ((double)gy - (double)ey);
        fz -= s.w * (kTwoPi / R.g.L[2]) * ((double)gz - (double)ez);
      } else {
        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll 4
        for (int l = 0; l < P; ++l) {
          const GatherMode gm = md[l];
          const double t = turn_fraction(gm.mx, gm.my, gm.mz, s.x, s.y, s.z);
          double sn, cs;
          sincos_turn_f64(t, &sn, &cs);
          const double g = gm.a * cs - gm.b * sn;
          gx = fma(g, gm.mx, gx);
          gy = fma(g, gm.my, gy);
          gz = fma(g, gm.mz, gz);
        }
        fx -= s.w * (kTwoPi / R.g.L[0]) * gx;
        fy -= s.w * (kTwoPi / R.g.L[1]) * gy;
        fz -= s.w * (kTwoPi / R.g.L[2]) * gz;
      }
    }
    a.ofx[i] = fx;
    a.ofy[i] = fy;
    a.ofz[i] = fz;
    if (a.mode == 0) {
      const double u = a.ovx[i] + a.h * fx, v = a.ovy[i] + a.h * fy, w = a.ovz[i] + a.h * fz;
      a.ovx[i] = u;
      a.ovy[i] = v;
      a.ovz[i] = w;
      if (!isfinite(u) || !isfinite(v) || !isfinite(w)) atomicOr(a.err, kErrNonFinite);
    } else {
      const int j = a.perm[i];
      a.cfx[j] = fx;
      a.cfy[j] = fy;
      a.cfz[j] = fz;
    }
  }
  if (a.mode == 0 && gtid == 0) *((volatile uint64_t *)a.eval) = eval + 1;
}

// The near field of every particle of the batch, between the two launches of
// the step kernel: a plain launch, so that its occupancy is not bound to the
// persistent kernel's registers. Four waves per SIMD in FP32C (no spills;
// five, with 13 VGPRs spilled, ran no faster), three in FP64 (16 VGPRs
// spilled, 11.0 against 12.1 ms per 256-replica step at two).
template <bool F32>
__global__ void __launch_bounds__(kBatchThreads) __attribute__((amdgpu_waves_per_eu(F32 ? 4 : 3)))
k_batch_near(BatchArgs a) {
  const int64_t i = blockIdx.x * (int64_t)kBatchThreads + threadIdx.x;
  if (i >= a.ntot) return;
  if (a.pp.do_coul || a.pp.do_lj) {
    batch_pair<F32>(a, a.reps[a.rep_of[i]], i);
  } else {
    a.ofx[i] = 0.0;
    a.ofy[i] = 0.0;
    a.ofz[i] = 0.0;
  }
}

int batch_grid_blocks(int prec, int device) {
  int per_cu = 0, cus = 0;
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
  if (prec == RBE_FP32C)
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_batch_step<true>),
                                                 kBatchThreads, 0);
  else
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void *>(k_batch_step<false>),
                                                 kBatchThreads, 0);
  if (per_cu < 1) per_cu = 1;
  if (cus < 1) cus = 1;
  return per_cu * cus;
}

void launch_batch_step(int prec, int blocks, const BatchArgs &a, hipStream_t st) {
  BatchArgs a1 = a, a2 = a;
  a1.launch_part = 1;
  a2.launch_part = 2;
  const unsigned near_blocks = (unsigned)((a.ntot + kBatchThreads - 1) / kBatchThreads);
  if (prec == RBE_FP32C) {
    k_batch_step<true><<<blocks, kBatchThreads, 0, st>>>(a1);
    k_batch_near<true><<<near_blocks, kBatchThreads, 0, st>>>(a);
    k_batch_step<true><<<blocks, kBatchThreads, 0, st>>>(a2);
  } else {
    k_batch_step<false><<<blocks, kBatchThreads, 0, st>>>(a1);
    k_batch_near<false><<<near_blocks, kBatchThreads, 0, st>>>(a);
    k_batch_step<false><<<blocks, kBatchThreads, 0, st>>>(a2);
  }
}

int batch_scan_tiles(int64_t nkeys) { return (int)((nkeys + kScanTileB - 1) / kScanTileB); }

hipError_t add_batch_node(hipGraph_t graph, hipGraphNode_t *node, const hipGraphNode_t *deps, int ndeps, int prec,
                          int blocks, BatchArgs *a) {
  const bool f32 = prec == RBE_FP32C;
  BatchArgs parts[3] = {*a, *a, *a};
  parts[0].launch_part = 1;
  parts[2].launch_part = 2;
  void *funcs[3] = {f32 ? reinterpret_cast<void *>(k_batch_step<true>) : reinterpret_cast<void *>(k_batch_step<false>),
                    f32 ? reinterpret_cast<void *>(k_batch_near<true>) : reinterpret_cast<void *>(k_batch_near<false>),
                    f32 ? reinterpret_cast<void *>(k_batch_step<true>) : reinterpret_cast<void *>(k_batch_step<false>)};
  const unsigned grids[3] = {(unsigned)blocks, (unsigned)((a->ntot + kBatchThreads - 1) / kBatchThreads),
                             (unsigned)blocks};
  hipGraphNode_t prev = nullptr;
  for (int k = 0; k < 3; ++k) {
    hipKernelNodeParams kp{};
    kp.func = funcs[k];
    kp.gridDim = dim3(grids[k]);
    kp.blockDim = dim3(kBatchThreads);
    kp.sharedMemBytes = 0;
    void *args[] = {&parts[k]};
    kp.kernelParams = args;
    kp.extra = nullptr;
    // the node copies the arguments
    const hipGraphNode_t dep = prev;
    const hipError_t e = k == 0 ? hipGraphAddKernelNode(&prev, graph, deps, (size_t)ndeps, &kp)
                                : hipGraphAddKernelNode(&prev, graph, &dep, 1, &kp);
    if (e != hipSuccess) return e;
  }
  *node = prev;
  return hipSuccess;
}

__global__ void __launch_bounds__(256) k_qstats_rep(const int64_t *__restrict__ off, const double *__restrict__ q,
                                                    int32_t *__restrict__ nq, double *__restrict__ qs) {
  __shared__ int lc[4];
  __shared__ double ls[4], la[4];
  const int r = blockIdx.x;
  const int64_t lo = off[r], hi = off[r + 1];
  int c = 0;
  double s = 0.0, a = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += 256) {
    const double v = q[i];
    c += v != 0.0;
    s += v;
    a += fabs(v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    c += __shfl_xor(c, o, 64);
    s += __shfl_xor(s, o, 64);
    a += __shfl_xor(a, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    lc[w] = c;
    ls[w] = s;
    la[w] = a;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    nq[r] = lc[0] + lc[1] + lc[2] + lc[3];
    qs[2 * r] = (ls[0] + ls[1]) + (ls[2] + ls[3]);
    qs[2 * r + 1] = (la[0] + la[1]) + (la[2] + la[3]);
  }
}

void launch_qstats_rep(int nrep, const int64_t *off, const double *q, int32_t *nq, double *qs, hipStream_t st) {
  k_qstats_rep<<<nrep, 256, 0, st>>>(off, q, nq, qs);
}

// Per-replica checks of Eq. 1 (flags kErrNonNeutral / kErrNonFinite) and the
// structure-factor layout of this call from the device counts: replica r's
// charged particles in chunks of chunk_len, its chunk partials at chunk_off,
// its (chunk, 64-mode group) items at rho_item_off; *rho_items receives the
// total, *bad_rep the first replica that failed a check (-1: none). One
// thread: the replica count is small.
__global__ void k_batch_layout(int nrep, const int32_t *__restrict__ nq, const double *__restrict__ qs, int groups,
                               int chunk_len, RepDesc *__restrict__ reps, int *__restrict__ rho_items,
                               int *__restrict__ bad_rep, int *err) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  int chunk_off = 0;
  int64_t items = 0;
  int flags = 0, bad = -1;
  for (int r = 0; r < nrep; ++r) {
    const double sq = qs[2 * r], sa = qs[2 * r + 1];
    int f = 0;
    if (!isfinite(sq) || !isfinite(sa)) f = kErrNonFinite;
    else if (fabs(sq) > 1e-10 * fmax(sa, 1e-300) && fabs(sq) > 1e-12) f = kErrNonNeutral;
    if (f && bad < 0) bad = r;
    flags |= f;
    RepDesc &d = reps[r];
    d.nq = nq[r];
    d.chunk_len = chunk_len;
    d.nchunks = (d.nq + chunk_len - 1) / chunk_len;
    d.chunk_off = chunk_off;
    d.rho_item_off = (int)items;
    chunk_off += d.nchunks;
    items += (int64_t)d.nchunks * groups;
  }
  *rho_items = (int)items;
  *bad_rep = bad;
  if (flags) atomicOr(err, flags);
}

void launch_batch_layout(int nrep, const int32_t *nq, const double *qs, int P, int chunk_len, RepDesc *reps,
                         int *rho_items, int *bad_rep, int *err, hipStream_t st) {
  k_batch_layout<<<1, 64, 0, st>>>(nrep, nq, qs, (P + 63) / 64, chunk_len, reps, rho_items, bad_rep, err);
}

__global__ void k_set_u64(uint64_t *p, uint64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

void launch_set_u64(uint64_t *p, uint64_t v, hipStream_t st) { k_set_u64<<<1, 64, 0, st>>>(p, v); }

}  // namespace rbe
