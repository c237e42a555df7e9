// Ghost shell of a subdomain (Sec. 2.3.2): copies of the native particles
// near a face, shifted by whole box edges, so the near-field kernels can
// treat the box as a padded, non-periodic region in which natives and ghosts
// share one traversal path.
//
// The shell is built directly in the padded grid's cell order. A padded cell
// P outside the native grid holds the images of the natives of its periodic
// source cell wrap(P), shifted by the box edges that take the source cell to
// P: the images a staged x, then y, then z exchange delivers into P when each
// stage forwards the earlier stages' ghosts (edge and corner cells receive
// their images by forwarding). The natives are already sorted by (species,
// cell), so the shell is a count per padded cell, a scan and a copy, and its
// records come out sorted. The layer is goff[d] cells thick, at least the
// ghost width: images beyond the ghost width but inside the layer are kept;
// they lie farther than every cutoff from every native, so the near field
// passes over them. Only positions, charges and ids are copied (the fields
// the near field reads); ghosts are never integrated.
#include "kernels.h"

namespace rbe {

// Padded key -> (species block, unwrapped cell relative to the native grid).
// Returns false for cells of the native grid (they hold no ghosts).
__device__ inline bool ghost_cell(const Grid &g, int64_t key, int *blk, int *x, int *y, int *z) {
  *blk = (int)(key / g.pncell);
  const int64_t p = key - (int64_t)*blk * g.pncell;
  *x = (int)(p % g.pnx) - g.goff[0];
  *y = (int)((p / g.pnx) % g.pny) - g.goff[1];
  *z = (int)(p / ((int64_t)g.pnx * g.pny)) - g.goff[2];
  return !(*x >= 0 && *x < g.nx && *y >= 0 && *y < g.ny && *z >= 0 && *z < g.nz);
}

// count[key] = natives of the source cell of ghost cell key (0 for native cells).
__global__ void __launch_bounds__(256) k_ghost_cell_counts(Grid g, const int32_t *__restrict__ cell_start,
                                                           int32_t *__restrict__ count) {
  const int64_t key = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (key >= 2 * (int64_t)g.pncell) return;
  int blk, x, y, z;
  int c = 0;
  if (ghost_cell(g, key, &blk, &x, &y, &z)) {
    const int wx = x - floor_div(x, g.nx) * g.nx, wy = y - floor_div(y, g.ny) * g.ny,
              wz = z - floor_div(z, g.nz) * g.nz;
    const int64_t src = (int64_t)blk * g.ncell + ((int64_t)wz * g.ny + wy) * g.nx + wx;
    c = cell_start[src + 1] - cell_start[src];
  }
  count[key] = c;
}

// Copies the shifted natives of each ghost cell's source cell to its slots
// and clamps the cell starts to the capacity (cells past it end up empty and
// the overflow is flagged), so no reader goes past the ghost arrays. One
// thread per padded key, plus one for the end entry.
__global__ void __launch_bounds__(256) k_ghost_fill(Grid g, int64_t cap, const int32_t *__restrict__ cell_start,
                                                    const double4 *__restrict__ xq, const int32_t *__restrict__ ids,
                                                    int32_t *__restrict__ gstart, double4 *__restrict__ gxq,
                                                    int32_t *__restrict__ gid, int32_t *__restrict__ gcount,
                                                    int *err) {
  const int64_t key = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nkeys = 2 * (int64_t)g.pncell;
  if (key > nkeys) return;
  const int64_t d0 = gstart[key];
  if (key == nkeys) {
    if (d0 > cap) atomicOr(err, kErrGhostOverflow);
    *gcount = (int32_t)(d0 < cap ? d0 : cap);
    gstart[key] = (int32_t)(d0 < cap ? d0 : cap);
    return;
  }
  int blk, x, y, z;
  if (ghost_cell(g, key, &blk, &x, &y, &z)) {
    const int qx = floor_div(x, g.nx), qy = floor_div(y, g.ny), qz = floor_div(z, g.nz);
    const int wx = x - qx * g.nx, wy = y - qy * g.ny, wz = z - qz * g.nz;
    const double sx = (double)qx * g.L[0], sy = (double)qy * g.L[1], sz = (double)qz * g.L[2];
    const int64_t src = (int64_t)blk * g.ncell + ((int64_t)wz * g.ny + wy) * g.nx + wx;
    int64_t d = d0;
    for (int j = cell_start[src]; j < cell_start[src + 1] && d < cap; ++j, ++d) {
      const double4 r = xq[j];
      gxq[d] = make_double4(r.x + sx, r.y + sy, r.z + sz, r.w);
      gid[d] = ids[j];
    }
  }
  gstart[key] = (int32_t)(d0 < cap ? d0 : cap);
}

void launch_build_ghosts(const Grid &g, int64_t n, const int32_t *cell_start, const Sorted &s,
                         const GhostBuffers &gb, int *err, hipStream_t st) {
  (void)n;
  const int64_t nkeys = 2 * (int64_t)g.pncell;
  const unsigned blocks = (unsigned)((nkeys + 255) / 256);
  k_ghost_cell_counts<<<blocks, 256, 0, st>>>(g, cell_start, gb.cell_count);
  launch_exclusive_scan(gb.cell_count, nkeys, gb.cell_start, gb.cell_scan_tmp, st);
  k_ghost_fill<<<(unsigned)((nkeys + 1 + 255) / 256), 256, 0, st>>>(g, gb.cap, cell_start, s.xq, s.id, gb.cell_start,
                                                                    gb.xq, gb.id, gb.count, err);
}

}  // namespace rbe
