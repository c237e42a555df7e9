// LJ sums of the FP32C form over LDS-staged cell tiles (Sec. 2.1, Eq. 8;
// Sec. 2.2 cell lists): every particle i of the launch's species blocks
// against every j (both species) with r <= r_lj, G_LJ(r) d. The charged
// particles' screened Coulomb terms are summed by the thread-form walks.
//
// A workgroup owns a tile of TX x TY x TZ cells. It stages the records of the
// tile's halo (the cells within the stencil of any own cell) in LDS once,
// converted to the tile's frame: FP32 coordinates relative to the tile's
// centre (the periodic image shift applied first, in FP64). Each thread then
// takes one particle i of the
// tile and walks the halo rows its reach sphere touches, each row trimmed to
// the x-cells the sphere spans, reading the candidates from LDS. Halo cells
// are met once per unwrapped cell index, i.e. once per (cell, periodic image),
// so no image is counted twice (the cutoffs are at most half the box).
//
// r^2 in FP32 from the frame coordinates; a pair whose r^2 lies within
// a relative band of 2^-16 around the cutoff is re-classified from the FP64
// records (minimum image), so cutoff membership is the FP64 one. The pair
// terms of a row are summed in FP32 and each row's sum is added to the total
// with Kahan compensation.
//
// A halo larger than the LDS staging is processed in chunks of whole rows
// (any density is handled; a single row beyond capacity is flagged).
#include "pair_device.h"

namespace rbe {

struct TileCtx {
  PairParams pp;
  int TX, TY, TZ;          // own cells per tile
  Sten s;                  // halo radius in cells
  int ntx, nty, ntz;       // tiles per axis
  int cap;                 // records the LDS staging holds
  int iblk;                // species blocks supplying i (bit 0 charged, bit 1 neutral)
  const double4 *__restrict__ xq;
  const int32_t *__restrict__ cell_start;
  const double4 *__restrict__ gxq;          // ghost shell (GHOST)
  const int32_t *__restrict__ gcell_start;
  int64_t n;                                // natives; ghost records are indexed from n on
  double *__restrict__ fx;
  double *__restrict__ fy;
  double *__restrict__ fz;
  unsigned long long *__restrict__ counters;  // [4] when counting
  int *err;
};

constexpr int kTileThreads = 256;
constexpr int kTileMaxSegs = 64;    // own row segments (rows x species blocks) of a tile
constexpr int kTileMaxChunks = 64;  // halo chunks of a tile whose halo exceeds the staging
constexpr int kTileIMax = 320;      // particles of a tile grouped by quadrant (more: cell order)

// A record of the LDS staging is a float4: the FP32 frame coordinates and,
// in w, the record's index as bits (the LJ terms need no charge).

// Records of one halo cell, in two sources per species block (natives and
// ghosts). Unwrapped cell (xc, yc, zc); returns the image shift (periodic).
struct CellSrc {
  int a[4], b[4];       // [natives blk 0, ghosts blk 0, natives blk 1, ghosts blk 1) ranges
  double sx, sy, sz;    // image shift (periodic traversal)
};

template <bool GHOST>
__device__ inline void cell_sources(const TileCtx &c, int xc, int yc, int zc, CellSrc *out) {
  const Grid &g = c.pp.g;
  for (int k = 0; k < 4; ++k) out->a[k] = out->b[k] = 0;
  out->sx = out->sy = out->sz = 0.0;
  if (GHOST) {
    const bool native = xc >= 0 && xc < g.nx && yc >= 0 && yc < g.ny && zc >= 0 && zc < g.nz;
    const int px = xc + g.goff[0], py = yc + g.goff[1], pz = zc + g.goff[2];
    const bool padded = px >= 0 && px < g.pnx && py >= 0 && py < g.pny && pz >= 0 && pz < g.pnz;
    for (int b = 0; b < 2; ++b) {
      if (native) {
        const int64_t key = (int64_t)b * g.ncell + ((int64_t)zc * g.ny + yc) * g.nx + xc;
        out->a[2 * b] = c.cell_start[key];
        out->b[2 * b] = c.cell_start[key + 1];
      }
      if (padded) {
        const int64_t key = (int64_t)b * g.pncell + ((int64_t)pz * g.pny + py) * g.pnx + px;
        out->a[2 * b + 1] = c.gcell_start[key];
        out->b[2 * b + 1] = c.gcell_start[key + 1];
      }
    }
  } else {
    const int qx = floor_div(xc, g.nx), qy = floor_div(yc, g.ny), qz = floor_div(zc, g.nz);
    const int wx = xc - qx * g.nx, wy = yc - qy * g.ny, wz = zc - qz * g.nz;
    out->sx = (double)qx * g.L[0];
    out->sy = (double)qy * g.L[1];
    out->sz = (double)qz * g.L[2];
    for (int b = 0; b < 2; ++b) {
      const int64_t key = (int64_t)b * g.ncell + ((int64_t)wz * g.ny + wy) * g.nx + wx;
      out->a[2 * b] = c.cell_start[key];
      out->b[2 * b] = c.cell_start[key + 1];
    }
  }
}

// Block-wide exclusive scan of v[0..m) in LDS (in place); returns the total.
__device__ inline int tile_scan(int *v, int m, int *wsum) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (m + kTileThreads - 1) / kTileThreads;
  const int lo = min(m, tid * per), hi = min(m, lo + per);
  int s = 0;
  for (int k = lo; k < hi; ++k) s += v[k];
  int incl = s;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) wsum[wave] = incl;
  __syncthreads();
  int off = 0, tot = 0;
  for (int w = 0; w < kTileThreads / 64; ++w) {
    if (w < wave) off += wsum[w];
    tot += wsum[w];
  }
  int run = off + incl - s;
  for (int k = lo; k < hi; ++k) {
    const int x = v[k];
    v[k] = run;
    run += x;
  }
  __syncthreads();
  return tot;
}

// Distance of p to the slab [lo, lo + h), less the margin, at least 0.
__device__ inline float tile_gap(float p, float lo, float h, float margin) {
  const float d = lo - p > 0.0f ? lo - p : (p - (lo + h) > 0.0f ? p - (lo + h) : 0.0f);
  return d > margin ? d - margin : 0.0f;
}

// LJ pair scalar without the cutoff test (the caller masks): the shape
// u (2 sigma^6 u - 1) / r^2 with u = r^-6, so that G_LJ(r) of Eq. 8 is
// 24 eps sigma^6 times it (the constant is applied once to the sum).
__device__ inline float lj_shape(float r2, float two_s6) {
  const float rinv2 = __builtin_amdgcn_rcpf(r2);
  const float u = rinv2 * rinv2 * rinv2;
  return u * fmaf(u, two_s6, -1.0f) * rinv2;
}

// s += v with Kahan compensation c.
__device__ inline void tile_kahan(float &s, float &c, float v) {
#pragma clang fp contract(off)
  const float y = v - c;
  const float t = s + y;
  c = (t - s) - y;
  s = t;
}

// Five waves per SIMD (at most 96 VGPRs, two of them spilled outside the
// candidate loop): 25.8 against 27.3 ms per 64M step at four.
template <bool GHOST, bool COUNT>
__global__ void __launch_bounds__(kTileThreads) __attribute__((amdgpu_waves_per_eu(5))) k_pair_tile(TileCtx c) {
  using T = float;
  using V = float4;
  extern __shared__ __align__(16) unsigned char tile_lds[];
  __shared__ int wsum[kTileThreads / 64];
  __shared__ int seg_n[kTileMaxSegs];       // own row segments: i count, then prefix
  __shared__ int seg_g0[kTileMaxSegs];      // first native index of each segment
  __shared__ int seg_i0[kTileMaxSegs + 1];
  __shared__ int chunk_r0[kTileMaxChunks], chunk_r1[kTileMaxChunks];  // row ranges staged together
  __shared__ int nchunk_s;
  __shared__ int ilist[kTileIMax];  // the tile's particles grouped by quadrant
  __shared__ int qcnt[4], qoff[4];

  const PairParams &pp = c.pp;
  const Grid &g = pp.g;
  const int tid = threadIdx.x;
  const int tile = (int)xcd_block(blockIdx.x, gridDim.x);
  const int tx = tile % c.ntx, ty = (tile / c.ntx) % c.nty, tz = tile / (c.ntx * c.nty);
  const int x0 = tx * c.TX, y0 = ty * c.TY, z0 = tz * c.TZ;
  const int HX = c.TX + 2 * c.s.x, HY = c.TY + 2 * c.s.y, HZ = c.TZ + 2 * c.s.z;
  const int nrows = HY * HZ, ncells = nrows * HX;
  const double hx = g.L[0] / g.nx, hy = g.L[1] / g.ny, hz = g.L[2] / g.nz;
  // frame: relative to the tile centre
  const double ox = (x0 + 0.5 * c.TX) * hx;
  const double oy = (y0 + 0.5 * c.TY) * hy;
  const double oz = (z0 + 0.5 * c.TZ) * hz;
  // low corner of the halo in the frame, cell edges and their inverse
  const T X0 = (T)((x0 - c.s.x) * hx - ox), Y0 = (T)((y0 - c.s.y) * hy - oy), Z0 = (T)((z0 - c.s.z) * hz - oz);
  const T Hy = (T)hy, Hz = (T)hz, invHx = (T)(1.0 / hx);
  const T margin = T(1e-4);
  const T rc2 = (T)pp.rlj2;
  const double rc2d = pp.rlj2;
  // FP32 classes of r^2 from its bits (non-negative floats order as their
  // bit patterns), lo = rc2 (1 - 2^-16), hi = rc2 (1 + 2^-16): with
  // d = bits(r^2) - 1 - bits(lo) (mod 2^32), d >= 2^32 - bits(lo) is
  // 0 < r^2 <= lo (r^2 = 0, the particle itself, wraps out of it), and
  // d < bits(hi) - bits(lo) is the guard band lo < r^2 <= hi, classified
  // from the FP64 records
  const T band = rc2 * T(1.52587890625e-05);
  const unsigned lo_bits = __float_as_uint(rc2 - band), hi_bits = __float_as_uint(rc2 + band);
  const unsigned d_off = ~lo_bits, in_min = 0u - lo_bits, band_w = hi_bits - lo_bits;
  // LJ: sigma^6 and the force constant 24 eps sigma^6 of the shape function
  const double s6 = pp.sig2 * pp.sig2 * pp.sig2;
  const T two_s6 = (T)(2.0 * s6);
  const double lj_scale = pp.eps24 * s6;

  // LDS: cell starts [ncells + 1], records [cap]
  int *cs = (int *)tile_lds;
  V *rec = (V *)(tile_lds + ((size_t)(ncells + 1) * sizeof(int) + 15) / 16 * 16);

  // ---- own row segments (one per own row and species block) ----------------
  const int nsegs = 2 * c.TY * c.TZ;
  if (tid < nsegs) {
    const int b = tid / (c.TY * c.TZ), rr = tid % (c.TY * c.TZ);
    const int yy = y0 + rr % c.TY, zz = z0 + rr / c.TY;
    const int xe = min(x0 + c.TX, g.nx);
    int a = 0, e = 0;
    if (((c.iblk >> b) & 1) && yy < g.ny && zz < g.nz && x0 < xe) {
      const int64_t key = (int64_t)b * g.ncell + ((int64_t)zz * g.ny + yy) * g.nx;
      a = c.cell_start[key + x0];
      e = c.cell_start[key + xe];
    }
    seg_n[tid] = e - a;
    seg_g0[tid] = a;
  }
  // ---- halo cell counts -----------------------------------------------------
  for (int h = tid; h < ncells; h += kTileThreads) {
    const int ix = h % HX, row = h / HX;
    CellSrc src;
    cell_sources<GHOST>(c, x0 - c.s.x + ix, y0 - c.s.y + row % HY, z0 - c.s.z + row / HY, &src);
    int cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt += src.b[k] - src.a[k];
    cs[h] = cnt;
  }
  __syncthreads();
  if (tid == 0) {
    int tot = 0;
    for (int k = 0; k < nsegs; ++k) {
      seg_i0[k] = tot;
      tot += seg_n[k];
    }
    seg_i0[nsegs] = tot;
  }
  const int total = tile_scan(cs, ncells, wsum);
  const int ni = seg_i0[nsegs];
  if (ni == 0) return;  // uniform: no particle of these species in the tile
  // chunks of whole rows that fit the staging (normally one); a single row
  // beyond the staging is left out (an empty chunk) and flagged
  if (tid == 0) {
    cs[ncells] = total;
    int nch = 0, row0 = 0;
    while (row0 < nrows && nch < kTileMaxChunks) {
      int r1 = row0;
      while (r1 < nrows && cs[(r1 + 1) * HX] - cs[row0 * HX] <= c.cap) ++r1;
      if (r1 == row0) {
        atomicOr(c.err, kErrTileOverflow);
        chunk_r0[nch] = chunk_r1[nch] = row0;
        r1 = row0 + 1;
      } else {
        chunk_r0[nch] = row0;
        chunk_r1[nch] = r1;
      }
      ++nch;
      row0 = r1;
    }
    if (row0 < nrows) atomicOr(c.err, kErrTileOverflow);
    nchunk_s = nch;
  }
  __syncthreads();
  const int nchunk = nchunk_s;

  auto stage = [&](int r0, int r1) {
    const int base = cs[r0 * HX];
    for (int h = r0 * HX + tid; h < r1 * HX; h += kTileThreads) {
      const int ix = h % HX, row = h / HX;
      CellSrc src;
      cell_sources<GHOST>(c, x0 - c.s.x + ix, y0 - c.s.y + row % HY, z0 - c.s.z + row / HY, &src);
      int d = cs[h] - base;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const bool ghost = GHOST && (k & 1);
        for (int j = src.a[k]; j < src.b[k]; ++j, ++d) {
          const double4 p = ghost ? c.gxq[j] : c.xq[j];
          const int gj = ghost ? (int)c.n + j : j;
          V v;
          v.x = (T)((p.x + src.sx) - ox);
          v.y = (T)((p.y + src.sy) - oy);
          v.z = (T)((p.z + src.sz) - oz);
          v.w = __int_as_float(gj);
          rec[d] = v;
        }
      }
    }
  };
  if (nchunk == 1) stage(chunk_r0[0], chunk_r1[0]);
  __syncthreads();

  // The tile's particles in cell order, regrouped by the quadrant of their
  // cell's y/z cross-section they sit in: the threads of a wave then have
  // similar distances to each stencil row, hence similar trimmed row
  // lengths, and fewer lanes idle while the longest row is walked. (Which
  // thread takes a particle does not change its result.)
  auto nth_particle = [&](int li) {
    int sgi = 0;
    while (sgi + 1 < nsegs && seg_i0[sgi + 1] <= li) ++sgi;
    return seg_g0[sgi] + (li - seg_i0[sgi]);
  };
  const bool grouped = ni <= kTileIMax;
  if (grouped) {
    if (tid < 4) qcnt[tid] = 0;
    __syncthreads();
    for (int li = tid; li < ni; li += kTileThreads) {
      const double4 p = c.xq[nth_particle(li)];
      const int qy = p.y - cell_coord(p.y, g.inv_h[1], g.ny) * hy >= 0.5 * hy;
      const int qz = p.z - cell_coord(p.z, g.inv_h[2], g.nz) * hz >= 0.5 * hz;
      atomicAdd(&qcnt[qy + 2 * qz], 1);
    }
    __syncthreads();
    if (tid == 0) {
      int o = 0;
      for (int q = 0; q < 4; ++q) {
        qoff[q] = o;
        o += qcnt[q];
      }
    }
    __syncthreads();
    for (int li = tid; li < ni; li += kTileThreads) {
      const int gi = nth_particle(li);
      const double4 p = c.xq[gi];
      const int qy = p.y - cell_coord(p.y, g.inv_h[1], g.ny) * hy >= 0.5 * hy;
      const int qz = p.z - cell_coord(p.z, g.inv_h[2], g.nz) * hz >= 0.5 * hz;
      ilist[atomicAdd(&qoff[qy + 2 * qz], 1)] = gi;
    }
    __syncthreads();
  }

  unsigned long long n_pairs = 0, n_cand = 0;
  const int rounds = (ni + kTileThreads - 1) / kTileThreads;
  for (int round = 0; round < rounds; ++round) {
    const int li = round * kTileThreads + tid;
    const bool active = li < ni;
    int gi = 0;
    if (active) gi = grouped ? ilist[li] : nth_particle(li);
    const double4 pi = c.xq[active ? gi : 0];
    const T xi = (T)(pi.x - ox), yi = (T)(pi.y - oy), zi = (T)(pi.z - oz);
    // i's halo cell (an own cell: clamped there, so every row index below
    // stays inside the halo)
    const int ix = min(max(cell_coord(pi.x, g.inv_h[0], g.nx) - (x0 - c.s.x), c.s.x), c.s.x + c.TX - 1);
    const int iy = min(max(cell_coord(pi.y, g.inv_h[1], g.ny) - (y0 - c.s.y), c.s.y), c.s.y + c.TY - 1);
    const int iz = min(max(cell_coord(pi.z, g.inv_h[2], g.nz) - (z0 - c.s.z), c.s.z), c.s.z + c.TZ - 1);
    T S[3] = {T(0), T(0), T(0)}, K[3] = {T(0), T(0), T(0)};
    for (int ch = 0; ch < nchunk; ++ch) {
      const int r0 = chunk_r0[ch], r1 = chunk_r1[ch];
      if (nchunk > 1) {
        __syncthreads();
        stage(r0, r1);
        __syncthreads();
      }
      if (!active || r0 == r1) continue;
      const int base = cs[r0 * HX];
      // one candidate: displacement, r^2 and its FP32 class
      struct Cand {
        T dx, dy, dz, r2;
        bool in, band;
      };
      auto prep = [&](const V &v) {
        Cand k;
        k.dx = xi - v.x;
        k.dy = yi - v.y;
        k.dz = zi - v.z;
        k.r2 = fmaf(k.dz, k.dz, fmaf(k.dy, k.dy, k.dx * k.dx));
        const unsigned d = __float_as_uint(k.r2) + d_off;
        k.in = d >= in_min;
        k.band = d < band_w;
        return k;
      };
      // near the cutoff: the class from the FP64 records (minimum image)
      auto fp64_in = [&](const V &v) {
        const int gj = __float_as_int(v.w);
        const double4 pj = gj < c.n ? c.xq[gj] : c.gxq[gj - c.n];
        const double ex = min_image(pi.x - pj.x, g.L[0]), ey = min_image(pi.y - pj.y, g.L[1]),
                     ez = min_image(pi.z - pj.z, g.L[2]);
        return sq_dist(ex, ey, ez) <= rc2d;
      };
      auto add = [&](const Cand &k, T &px, T &py, T &pz) {
        T f = lj_shape(k.r2, two_s6);
        f = k.in ? f : T(0);
        px = fmaf(f, k.dx, px);
        py = fmaf(f, k.dy, py);
        pz = fmaf(f, k.dz, pz);
        if (COUNT) {
          ++n_cand;
          n_pairs += k.in;
        }
      };
      auto cand = [&](const V &v, T &px, T &py, T &pz) {
        Cand k = prep(v);
        if (k.band) k.in = fp64_in(v);
        add(k, px, py, pz);
      };
      // the rows the reach sphere touches, each trimmed to the x-cells it
      // spans; a row's terms are summed in FP32 and its sum added to the
      // total with Kahan compensation
      for (int dz = -c.s.z; dz <= c.s.z; ++dz) {
        const int rz = iz + dz;
        const T gz = tile_gap(zi, Z0 + (T)rz * Hz, Hz, margin);
        if (gz * gz > rc2) continue;
        for (int dy = -c.s.y; dy <= c.s.y; ++dy) {
          const int ry = iy + dy;
          const int row = rz * HY + ry;
          if (row < r0 || row >= r1) continue;
          const T gy = tile_gap(yi, Y0 + (T)ry * Hy, Hy, margin);
          const T rem = rc2 - (gy * gy + gz * gz);
          if (rem < T(0)) continue;
          // the hardware square root (within 1 ulp) suffices: the margin
          // (1e-4 in FP32) covers its error many times over
          const T ext = __builtin_amdgcn_sqrtf(rem) + margin;
          int xa = (int)floor((xi - ext - X0) * invHx), xb = (int)floor((xi + ext - X0) * invHx);
          xa = max(xa, max(ix - c.s.x, 0));
          xb = min(xb, min(ix + c.s.x, HX - 1));
          if (xa > xb) continue;
          const int ka = cs[row * HX + xa] - base, kb = cs[row * HX + xb + 1] - base;
          T px = T(0), py = T(0), pz = T(0);
          // four candidates per trip, all records requested before use; the
          // trip count runs on the record pointer alone
          const V *q = rec + ka;
          const V *const qe = rec + kb, *const qe4 = qe - 3;
          for (; q < qe4; q += 4) {
            const V v0 = q[0], v1 = q[1], v2 = q[2], v3 = q[3];
            Cand k0 = prep(v0), k1 = prep(v1), k2 = prep(v2), k3 = prep(v3);
            // one wave-uniform branch for the rare guard-band candidates of
            // the trip (the lane masks are combined as scalars)
            if (__builtin_amdgcn_ballot_w64(k0.band) | __builtin_amdgcn_ballot_w64(k1.band) |
                __builtin_amdgcn_ballot_w64(k2.band) | __builtin_amdgcn_ballot_w64(k3.band)) {
              if (k0.band) k0.in = fp64_in(v0);
              if (k1.band) k1.in = fp64_in(v1);
              if (k2.band) k2.in = fp64_in(v2);
              if (k3.band) k3.in = fp64_in(v3);
            }
            add(k0, px, py, pz);
            add(k1, px, py, pz);
            add(k2, px, py, pz);
            add(k3, px, py, pz);
          }
          if (q + 1 < qe) {
            const V v0 = q[0], v1 = q[1];
            cand(v0, px, py, pz);
            cand(v1, px, py, pz);
            q += 2;
          }
          if (q < qe) cand(q[0], px, py, pz);
          tile_kahan(S[0], K[0], px);
          tile_kahan(S[1], K[1], py);
          tile_kahan(S[2], K[2], pz);
        }
      }
    }
    if (active) {
      c.fx[gi] = lj_scale * ((double)S[0] - (double)K[0]);
      c.fy[gi] = lj_scale * ((double)S[1] - (double)K[1]);
      c.fz[gi] = lj_scale * ((double)S[2] - (double)K[2]);
    }
  }
  if (COUNT) {
    atomicAdd(&c.counters[1], n_pairs);
    atomicAdd(&c.counters[2], n_cand);
  }
}

// ---------------------------------------------------------------------------
// launch
// ---------------------------------------------------------------------------
constexpr size_t kTileLdsBytes = 48 * 1024;

// Tile of the LJ pass: y/z extent of about 4-5 sigma, x extent such that a
// tile holds about one particle per thread at the mean density, and its halo
// stays within the LDS staging (the staging is sized for the halo of the
// mean density with room to spare; denser halos are processed in chunks).
static void tile_geometry(const PairParams &pp, const Sten &s, int64_t n, TileCtx *c) {
  const Grid &g = pp.g;
  const double hyz = std::fmax(g.L[1] / g.ny, g.L[2] / g.nz);
  const int T = hyz >= 2.0 ? 2 : 4;  // 2 T^2 own row segments <= kTileMaxSegs
  c->TY = std::min(T, g.ny);
  c->TZ = std::min(T, g.nz);
  c->s = s;
  const double dens = (double)n / (double)g.ncell;  // records per cell (both species)
  const int HYZ = (c->TY + 2 * s.y) * (c->TZ + 2 * s.z);
  int tx = (int)(kTileThreads / std::fmax(dens * c->TY * c->TZ, 1e-9));
  tx = std::max(1, std::min(tx, g.nx));
  // the FP32 frame spans at most about 10 sigma either side of the tile centre
  const double hx = g.L[0] / g.nx;
  tx = std::max(1, std::min(tx, (int)(2.0 * (10.0 / hx - s.x))));
  // records of the mean halo within 60 % of the most the staging may hold
  auto cap_of = [&](int t) {
    const int ncells = HYZ * (t + 2 * s.x);
    const size_t fixed = ((size_t)(ncells + 1) * sizeof(int) + 15) / 16 * 16;
    return fixed >= kTileLdsBytes ? 0 : (int)((kTileLdsBytes - fixed) / sizeof(float4));
  };
  while (tx > 1 && 0.6 * cap_of(tx) < dens * HYZ * (tx + 2 * s.x)) --tx;
  c->TX = tx;
  // the staging holds the mean halo with 15 % and 64 records of headroom
  // (6-7 standard deviations of a Poisson halo count of this size); denser
  // halos go in chunks. A block then takes about 31 KB of LDS at the
  // subdomain's density, so that five blocks share a CU (the five waves per
  // SIMD the kernel is compiled for)
  const int want = (int)std::ceil(1.15 * dens * HYZ * (tx + 2 * s.x)) + 64;
  c->cap = std::min(cap_of(tx), std::max(want, 256));
  c->ntx = (g.nx + c->TX - 1) / c->TX;
  c->nty = (g.ny + c->TY - 1) / c->TY;
  c->ntz = (g.nz + c->TZ - 1) / c->TZ;
}

template <bool GHOST>
static void launch_tile_t(const TileCtx &c, hipStream_t st) {
  const int ncells = (c.TY + 2 * c.s.y) * (c.TZ + 2 * c.s.z) * (c.TX + 2 * c.s.x);
  const size_t lds = ((size_t)(ncells + 1) * sizeof(int) + 15) / 16 * 16 + (size_t)c.cap * sizeof(float4);
  const unsigned tiles = (unsigned)((int64_t)c.ntx * c.nty * c.ntz);
  if (c.counters)
    k_pair_tile<GHOST, true><<<tiles, kTileThreads, lds, st>>>(c);
  else
    k_pair_tile<GHOST, false><<<tiles, kTileThreads, lds, st>>>(c);
}

bool lj_tile_applicable(int prec, const PairParams &pp, int64_t n) {
  if (prec != RBE_FP32C || !pp.do_lj || n <= 0) return false;
  TileCtx c{};
  tile_geometry(pp, pp.s_lj, n, &c);
  const double dens = (double)n / (double)pp.g.ncell;
  const Grid &g = pp.g;
  // rows about as wide as the LJ reach (wider rows waste most candidates);
  // a halo row of the mean density fills at most an eighth of the staging,
  // so only rows far denser than the mean need a chunk of their own
  const double hyz = std::fmax(g.L[1] / g.ny, g.L[2] / g.nz);
  return hyz <= 1.2 * std::sqrt(pp.rlj2) && c.cap >= 512 && dens * (c.TX + 2 * c.s.x) <= c.cap / 8.0;
}

void launch_lj_tile(const PairParams &pp, int64_t n, int iblk, const Sorted &s, const int32_t *cell_start,
                    const GhostBuffers *gb, double *fx, double *fy, double *fz, unsigned long long *counters,
                    int *err, hipStream_t st) {
  if (n <= 0) return;
  TileCtx c{};
  c.pp = pp;
  c.iblk = iblk;
  c.xq = s.xq;
  c.cell_start = cell_start;
  c.gxq = gb ? gb->xq : nullptr;
  c.gcell_start = gb ? gb->cell_start : nullptr;
  c.n = n;
  c.fx = fx;
  c.fy = fy;
  c.fz = fz;
  c.counters = counters;
  c.err = err;
  tile_geometry(pp, pp.s_lj, n, &c);
  if (gb) launch_tile_t<true>(c, st);
  else launch_tile_t<false>(c, st);
}

}  // namespace rbe
