// Cell binning: stable counting sort of particles by (species, cell), and
// the reorder of the particle arrays into that order (Sec. 2.2: linked-cell
// reassignment and cell-wise reordering).
//
// key = s * C + (c_z n_y + c_y) n_x + c_x with s = 0 for charged and 1 for
// neutral particles. Charged particles therefore occupy one contiguous range
// [0, start[C]) in cell order, which the Fourier kernels walk directly.
//
// Steps: keys + histogram (integer atomics give exact counts) -> exclusive
// scan -> provisional scatter (atomic slot order, not deterministic) ->
// stable placement: each bucket's entries (input indices) are put in
// increasing order, so a particle's final slot is start[key] + the number of
// bucket members with a smaller input index. The output is a pure function
// of the input, whatever order the atomics took.
//
// The input of a step is the previous step's cell order, so equal keys come
// in runs. A wave takes one atomic per run (its length) and hands out the
// slots of the run in input order; a bucket is then usually already in order
// and its placement a copy (checked per bucket; out-of-order buckets are
// sorted by insertion).
#include "rbe_internal.h"
#include "kernels.h"

namespace rbe {

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_i32<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

void launch_fill_f64(double *p, int64_t n, double v, hipStream_t st) {
  if (n <= 0) return;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_f64<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
}

// ---------------------------------------------------------------------------
// keys + histogram
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_bin_keys(int64_t n, const double *__restrict__ x, const double *__restrict__ y,
                                                  const double *__restrict__ z, const double *__restrict__ q, Grid g,
                                                  int32_t *__restrict__ key, int32_t *__restrict__ slot,
                                                  int32_t *__restrict__ count) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = i < n;
  int k = -1 - (int)(threadIdx.x & 63);  // lanes past the end: a key no other lane has
  if (active) {
    const int cx = cell_coord(wrap_coord(x[i], g.L[0]), g.inv_h[0], g.nx);
    const int cy = cell_coord(wrap_coord(y[i], g.L[1]), g.inv_h[1], g.ny);
    const int cz = cell_coord(wrap_coord(z[i], g.L[2]), g.inv_h[2], g.nz);
    k = (q[i] == 0.0 ? g.ncell : 0) + (cz * g.ny + cy) * g.nx + cx;
    key[i] = k;
  }
  const int sl = run_slot(k, active, count);  // every lane of the wave takes part in the vote
  if (active) slot[i] = sl;
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 counts (three phases)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

// Block-wide exclusive scan of one value per thread; returns the block total.
__device__ inline int block_exclusive_scan(int v, int *lds_waves, int *out_excl) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane == 63) lds_waves[wave] = incl;
  __syncthreads();
  int wave_off = 0, total = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    const int s = lds_waves[w];
    if (w < wave) wave_off += s;
    total += s;
  }
  __syncthreads();
  *out_excl = wave_off + incl - v;
  return total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_tiles(const int32_t *__restrict__ cnt, int64_t n,
                                                              int32_t *__restrict__ tile_sum) {
  __shared__ int lds[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < n) s += cnt[base + k];
  int excl;
  const int total = block_exclusive_scan(s, lds, &excl);
  if (threadIdx.x == 0) tile_sum[blockIdx.x] = total;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_top(int32_t *__restrict__ tile_sum, int64_t ntiles,
                                                            int32_t *__restrict__ grand_total) {
  __shared__ int lds[kScanThreads / 64];
  int carry = 0;
  for (int64_t b = 0; b < ntiles; b += kScanThreads) {
    const int64_t i = b + threadIdx.x;
    const int v = i < ntiles ? tile_sum[i] : 0;
    int excl;
    const int total = block_exclusive_scan(v, lds, &excl);
    if (i < ntiles) tile_sum[i] = carry + excl;
    carry += total;
  }
  if (threadIdx.x == 0) *grand_total = carry;
}

__global__ void __launch_bounds__(kScanThreads) k_scan_apply(const int32_t *__restrict__ cnt, int64_t n,
                                                              const int32_t *__restrict__ tile_off,
                                                              int32_t *__restrict__ start) {
  __shared__ int lds[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int v[kScanItems];
  int s = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    v[k] = base + k < n ? cnt[base + k] : 0;
    s += v[k];
  }
  int excl;
  block_exclusive_scan(s, lds, &excl);
  int run = tile_off[blockIdx.x] + excl;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    if (base + k < n) start[base + k] = run;
    run += v[k];
  }
}

int64_t scan_tiles(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// start[0..n] = exclusive scan of cnt[0..n); start[n] = total. tmp needs scan_tiles(n) ints.
void launch_exclusive_scan(const int32_t *cnt, int64_t n, int32_t *start, int32_t *tmp, hipStream_t st) {
  const int64_t nt = scan_tiles(n);
  k_scan_tiles<<<(unsigned)nt, kScanThreads, 0, st>>>(cnt, n, tmp);
  k_scan_top<<<1, kScanThreads, 0, st>>>(tmp, nt, start + n);
  k_scan_apply<<<(unsigned)nt, kScanThreads, 0, st>>>(cnt, n, tmp, start);
}

// ---------------------------------------------------------------------------
// provisional scatter and stable placement
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_scatter_prov(int64_t n, const int32_t *__restrict__ key,
                                                      const int32_t *__restrict__ slot,
                                                      const int32_t *__restrict__ start, int32_t *__restrict__ tmp) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  tmp[start[key[i]] + slot[i]] = (int32_t)i;
}

__global__ void __launch_bounds__(256) k_place_buckets(int64_t nkeys, const int32_t *__restrict__ start,
                                                       const int32_t *__restrict__ tmp, int32_t *__restrict__ perm) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= nkeys) return;
  place_bucket(start[k], start[k + 1], tmp, perm);
}

void launch_bin_clear(const BinBuffers &b, const Grid &g, hipStream_t st) {
  launch_fill_i32(b.count, 2 * (int64_t)g.ncell, 0, st);
}

void launch_bin_place(const BinBuffers &b, const Grid &g, int64_t n, int32_t *cell_start, int32_t *perm,
                      hipStream_t st) {
  const int64_t nkeys = 2 * (int64_t)g.ncell;
  launch_exclusive_scan(b.count, nkeys, cell_start, b.scan_tmp, st);
  if (n > 0) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_scatter_prov<<<blocks, 256, 0, st>>>(n, b.key, b.slot, cell_start, b.tmp);
    k_place_buckets<<<(unsigned)((nkeys + 255) / 256), 256, 0, st>>>(nkeys, cell_start, b.tmp, perm);
  }
}

void launch_bin(const BinBuffers &b, const Grid &g, int64_t n, const double *x, const double *y, const double *z,
                const double *q, int32_t *cell_start, int32_t *perm, hipStream_t st) {
  launch_bin_clear(b, g, st);
  if (n > 0) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_bin_keys<<<blocks, 256, 0, st>>>(n, x, y, z, q, g, b.key, b.slot, b.count);
  }
  launch_bin_place(b, g, n, cell_start, perm, st);
}

}  // namespace rbe
