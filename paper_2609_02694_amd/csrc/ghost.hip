// Ghost shell of a subdomain (Sec. 2.3.2): copies of the native particles
// that lie within the ghost width w of a face, shifted by one box edge, so
// the near-field kernels can treat the box as a padded, non-periodic region
// in which natives and ghosts share one traversal path.
//
// Copies are made direction by direction (x, then y, then z). Each stage
// marks the sources near the two faces of its axis, scans the marks, and
// appends the shifted copies; a stage's sources are the natives plus every
// ghost made by the earlier stages, so edge and corner images arrive by
// forwarding without diagonal copies. Only positions, charges and ids are
// copied (the fields the near field reads); ghosts are never integrated.
//
// The ghosts are then sorted by (species, padded cell) with the same stable
// counting sort as the natives, on the padded grid.
#include "kernels.h"

namespace rbe {

__device__ inline double rec_coord(const double4 &r, int d) { return d == 0 ? r.x : (d == 1 ? r.y : r.z); }

// flags[s] = 1 when source s lies within w of a face of axis d. Sources:
// s < n are native records, n <= s < n + G the ghosts made so far.
__global__ void __launch_bounds__(256) k_ghost_mark(int d, int64_t n, int64_t len, const double4 *__restrict__ xq,
                                                    const double4 *__restrict__ graw,
                                                    const int32_t *__restrict__ gcount, double L, double w,
                                                    int32_t *__restrict__ flags) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= len) return;
  int f = 0;
  const int64_t G = *gcount;
  if (s < n || s - n < G) {
    const double c = rec_coord(s < n ? xq[s] : graw[s - n], d);
    f = (c < w || c >= L - w) ? 1 : 0;
  }
  flags[s] = f;
}

// Appends the shifted copy of every marked source at G + offs[s].
__global__ void __launch_bounds__(256) k_ghost_copy(int d, int64_t n, int64_t len, int64_t cap,
                                                    const double4 *__restrict__ xq, const int32_t *__restrict__ ids,
                                                    double4 *__restrict__ graw, int32_t *__restrict__ gid,
                                                    const int32_t *__restrict__ gcount,
                                                    const int32_t *__restrict__ flags,
                                                    const int32_t *__restrict__ offs, double L, double w, int *err) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= len || !flags[s]) return;
  const int64_t dst = (int64_t)*gcount + offs[s];
  if (dst >= cap) {
    atomicOr(err, kErrGhostOverflow);
    return;
  }
  double4 r = s < n ? xq[s] : graw[s - n];
  const int32_t id = s < n ? ids[s] : gid[s - n];
  const double c = rec_coord(r, d);
  const double shifted = c < w ? c + L : c - L;
  if (d == 0) r.x = shifted;
  else if (d == 1) r.y = shifted;
  else r.z = shifted;
  graw[dst] = r;
  gid[dst] = id;
}

__global__ void k_ghost_count_add(int32_t *gcount, const int32_t *total, int64_t cap) {
  const int64_t v = (int64_t)*gcount + *total;
  *gcount = (int32_t)(v < cap ? v : cap);
}

// Padded cell index along one axis: goff + floor(x * inv_h), clamped to the
// padded grid (a NaN lands in cell 0).
__device__ inline int padded_coord(double x, double inv_h, int off, int pn) {
  const double t = floor(x * inv_h) + (double)off;
  if (t >= 0.0 && t < (double)pn) return (int)t;
  return t >= (double)pn ? pn - 1 : 0;
}

__global__ void __launch_bounds__(256) k_ghost_keys(int64_t cap, const int32_t *__restrict__ gcount,
                                                    const double4 *__restrict__ graw, Grid g,
                                                    int32_t *__restrict__ key, int32_t *__restrict__ slot,
                                                    int32_t *__restrict__ count) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= cap || k >= *gcount) return;
  const double4 r = graw[k];
  const int cx = padded_coord(r.x, g.inv_h[0], g.goff[0], g.pnx);
  const int cy = padded_coord(r.y, g.inv_h[1], g.goff[1], g.pny);
  const int cz = padded_coord(r.z, g.inv_h[2], g.goff[2], g.pnz);
  const int kk = (r.w == 0.0 ? g.pncell : 0) + (cz * g.pny + cy) * g.pnx + cx;
  key[k] = kk;
  slot[k] = atomicAdd(&count[kk], 1);
}

__global__ void __launch_bounds__(256) k_ghost_scatter(int64_t cap, const int32_t *__restrict__ gcount,
                                                       const int32_t *__restrict__ key,
                                                       const int32_t *__restrict__ slot,
                                                       const int32_t *__restrict__ start, int32_t *__restrict__ tmp) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= cap || k >= *gcount) return;
  tmp[start[key[k]] + slot[k]] = (int32_t)k;
}

// Stable placement and gather in one pass: slot = start[key] + number of
// bucket members with a smaller ghost index.
__global__ void __launch_bounds__(256) k_ghost_place(int64_t cap, const int32_t *__restrict__ gcount,
                                                     const int32_t *__restrict__ key,
                                                     const int32_t *__restrict__ start,
                                                     const int32_t *__restrict__ tmp,
                                                     const double4 *__restrict__ graw,
                                                     const int32_t *__restrict__ gid_raw, double4 *__restrict__ gxq,
                                                     int32_t *__restrict__ gid) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= cap || k >= *gcount) return;
  const int b = key[k];
  const int lo = start[b], hi = start[b + 1];
  int rank = 0;
  for (int t = lo; t < hi; ++t) rank += tmp[t] < (int32_t)k;
  gxq[lo + rank] = graw[k];
  gid[lo + rank] = gid_raw[k];
}

void launch_build_ghosts(const Grid &g, int64_t n, const Sorted &s, const GhostBuffers &gb, int *err,
                         hipStream_t st) {
  launch_fill_i32(gb.count, 1, 0, st);
  const double w = g.ghost_width;
  for (int d = 0; d < 3; ++d) {
    // stage 0 reads the natives only; later stages also the ghosts made so far
    const int64_t len = d == 0 ? n : n + gb.cap;
    if (len <= 0) continue;
    const unsigned blocks = (unsigned)((len + 255) / 256);
    k_ghost_mark<<<blocks, 256, 0, st>>>(d, n, len, s.xq, gb.raw_xq, gb.count, g.L[d], w, gb.flags);
    launch_exclusive_scan(gb.flags, len, gb.offs, gb.scan_tmp, st);
    k_ghost_copy<<<blocks, 256, 0, st>>>(d, n, len, gb.cap, s.xq, s.id, gb.raw_xq, gb.raw_id, gb.count, gb.flags,
                                         gb.offs, g.L[d], w, err);
    k_ghost_count_add<<<1, 1, 0, st>>>(gb.count, gb.offs + len, gb.cap);
  }
  // sort by (species, padded cell)
  const int64_t nkeys = 2 * (int64_t)g.pncell;
  launch_fill_i32(gb.cell_count, nkeys, 0, st);
  const unsigned cblocks = (unsigned)((gb.cap + 255) / 256);
  k_ghost_keys<<<cblocks, 256, 0, st>>>(gb.cap, gb.count, gb.raw_xq, g, gb.key, gb.slot, gb.cell_count);
  launch_exclusive_scan(gb.cell_count, nkeys, gb.cell_start, gb.cell_scan_tmp, st);
  k_ghost_scatter<<<cblocks, 256, 0, st>>>(gb.cap, gb.count, gb.key, gb.slot, gb.cell_start, gb.tmp);
  k_ghost_place<<<cblocks, 256, 0, st>>>(gb.cap, gb.count, gb.key, gb.cell_start, gb.tmp, gb.raw_xq, gb.raw_id,
                                         gb.xq, gb.id);
}

}  // namespace rbe
