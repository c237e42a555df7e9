// Ghost shell of a subdomain (Sec. 2.3.2): copies of the native particles
// that lie within the ghost width w of a face, shifted by one box edge, so
// the near-field kernels can treat the box as a padded, non-periodic region
// in which natives and ghosts share one traversal path.
//
// The images are those of a staged exchange x, then y, then z in which each
// stage also forwards the ghosts of the earlier stages (edge and corner
// images arrive by forwarding). A native within w of a face on a set A of
// axes (at most one face per axis, since w <= L/2) therefore has one image
// per non-empty subset of A, shifted by one box edge along each axis of the
// subset; they are made in one pass: count (2^|A| - 1) per native, scan,
// write. Only positions, charges and ids are copied (the fields the near
// field reads); ghosts are never integrated.
//
// The ghosts are then sorted by (species, padded cell) with the same stable
// counting sort as the natives, on the padded grid.
#include "kernels.h"

namespace rbe {

// Face bits of a native: bit d set when coordinate d lies within w of a
// face of axis d.
__device__ inline int face_bits(const double4 &r, const Grid &g, double w) {
  int f = 0;
  if (r.x < w || r.x >= g.L[0] - w) f |= 1;
  if (r.y < w || r.y >= g.L[1] - w) f |= 2;
  if (r.z < w || r.z >= g.L[2] - w) f |= 4;
  return f;
}

// counts[s] = number of images of native s (2^|A| - 1).
__global__ void __launch_bounds__(256) k_ghost_count(int64_t n, const double4 *__restrict__ xq, Grid g, double w,
                                                     int32_t *__restrict__ counts) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  counts[s] = (1 << __popc(face_bits(xq[s], g, w))) - 1;
}

// Writes the images of native s at offs[s] onwards, subsets in increasing
// bit order (x, y, xy, z, xz, yz, xyz).
__global__ void __launch_bounds__(256) k_ghost_emit(int64_t n, int64_t cap, const double4 *__restrict__ xq,
                                                    const int32_t *__restrict__ ids, Grid g, double w,
                                                    const int32_t *__restrict__ offs, double4 *__restrict__ graw,
                                                    int32_t *__restrict__ gid, int *err) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (s >= n) return;
  const double4 r = xq[s];
  const int f = face_bits(r, g, w);
  if (f == 0) return;
  // shifted coordinate of each axis (low face: +L, high face: -L)
  const double sx = r.x < w ? r.x + g.L[0] : r.x - g.L[0];
  const double sy = r.y < w ? r.y + g.L[1] : r.y - g.L[1];
  const double sz = r.z < w ? r.z + g.L[2] : r.z - g.L[2];
  int64_t dst = offs[s];
  for (int sub = 1; sub < 8; ++sub) {
    if ((sub & f) != sub) continue;
    if (dst < 0 || dst >= cap) {
      atomicOr(err, kErrGhostOverflow);
      return;
    }
    graw[dst] = make_double4((sub & 1) ? sx : r.x, (sub & 2) ? sy : r.y, (sub & 4) ? sz : r.z, r.w);
    gid[dst] = ids[s];
    ++dst;
  }
}

// ghost count = min(total images, capacity)
__global__ void k_ghost_total(int32_t *gcount, const int32_t *total, int64_t cap) {
  const int64_t v = *total;
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
  const int64_t n = min(cap, (int64_t)*gcount);
  if (k - (threadIdx.x & 63) >= n) return;  // whole wave past the end
  const bool active = k < n;
  int kk = -1 - (int)(threadIdx.x & 63);  // lanes past the end: a key no other lane has
  if (active) {
    const double4 r = graw[k];
    const int cx = padded_coord(r.x, g.inv_h[0], g.goff[0], g.pnx);
    const int cy = padded_coord(r.y, g.inv_h[1], g.goff[1], g.pny);
    const int cz = padded_coord(r.z, g.inv_h[2], g.goff[2], g.pnz);
    kk = (r.w == 0.0 ? g.pncell : 0) + (cz * g.pny + cy) * g.pnx + cx;
    key[k] = kk;
  }
  const int sl = run_slot(kk, active, count);  // every lane of the wave takes part
  if (active) slot[k] = sl;
}

__global__ void __launch_bounds__(256) k_ghost_scatter(int64_t cap, const int32_t *__restrict__ gcount,
                                                       const int32_t *__restrict__ key,
                                                       const int32_t *__restrict__ slot,
                                                       const int32_t *__restrict__ start, int32_t *__restrict__ tmp) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= cap || k >= *gcount) return;
  tmp[start[key[k]] + slot[k]] = (int32_t)k;
}

// Stable placement per bucket (entries in increasing creation order), then
// the gather of the records into that order.
__global__ void __launch_bounds__(256) k_ghost_buckets(int64_t nkeys, const int32_t *__restrict__ start,
                                                       const int32_t *__restrict__ tmp, int32_t *__restrict__ perm) {
  const int64_t b = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (b >= nkeys) return;
  place_bucket(start[b], start[b + 1], tmp, perm);
}

__global__ void __launch_bounds__(256) k_ghost_gather(int64_t cap, const int32_t *__restrict__ gcount,
                                                      const int32_t *__restrict__ perm,
                                                      const double4 *__restrict__ graw,
                                                      const int32_t *__restrict__ gid_raw, double4 *__restrict__ gxq,
                                                      int32_t *__restrict__ gid) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= cap || t >= *gcount) return;
  const int k = perm[t];
  gxq[t] = graw[k];
  gid[t] = gid_raw[k];
}

void launch_build_ghosts(const Grid &g, int64_t n, const Sorted &s, const GhostBuffers &gb, int *err,
                         hipStream_t st) {
  launch_fill_i32(gb.count, 1, 0, st);
  const double w = g.ghost_width;
  if (n > 0) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_ghost_count<<<blocks, 256, 0, st>>>(n, s.xq, g, w, gb.flags);
    launch_exclusive_scan(gb.flags, n, gb.offs, gb.scan_tmp, st);
    k_ghost_emit<<<blocks, 256, 0, st>>>(n, gb.cap, s.xq, s.id, g, w, gb.offs, gb.raw_xq, gb.raw_id, err);
    k_ghost_total<<<1, 1, 0, st>>>(gb.count, gb.offs + n, gb.cap);
  }
  // sort by (species, padded cell)
  const int64_t nkeys = 2 * (int64_t)g.pncell;
  launch_fill_i32(gb.cell_count, nkeys, 0, st);
  const unsigned cblocks = (unsigned)((gb.cap + 255) / 256);
  k_ghost_keys<<<cblocks, 256, 0, st>>>(gb.cap, gb.count, gb.raw_xq, g, gb.key, gb.slot, gb.cell_count);
  launch_exclusive_scan(gb.cell_count, nkeys, gb.cell_start, gb.cell_scan_tmp, st);
  k_ghost_scatter<<<cblocks, 256, 0, st>>>(gb.cap, gb.count, gb.key, gb.slot, gb.cell_start, gb.tmp);
  // the keys are no longer needed: their array receives the placement
  k_ghost_buckets<<<(unsigned)((nkeys + 255) / 256), 256, 0, st>>>(nkeys, gb.cell_start, gb.tmp, gb.key);
  k_ghost_gather<<<cblocks, 256, 0, st>>>(gb.cap, gb.count, gb.key, gb.raw_xq, gb.raw_id, gb.xq, gb.id);
}

}  // namespace rbe
