// Internal declarations of the RBE library (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/rbe.h"

namespace rbe {

constexpr double kPi = 3.14159265358979323846264338327950288;
constexpr double kTwoPi = 6.28318530717958647692528676655900577;

// ---------------------------------------------------------------------------
// Counter-based generators (definitions restated in include/rbe.h)
// ---------------------------------------------------------------------------
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ULL;   // SplitMix64 increment
constexpr uint64_t kTagModes = 0x4B4D4F4445534554ULL; // stream tag of the mode sample
constexpr uint64_t kTagShell = 0x52424C5348454C4CULL; // stream tag of the shell batches

__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
// Output n (0-based) of the SplitMix64 stream seeded by s.
__host__ __device__ inline uint64_t stream_out(uint64_t s, uint64_t n) { return mix64(s + (n + 1) * kGamma); }
__host__ __device__ inline double unit53(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

// lowbias32 (Wellons) and its inverse: bijections of 32-bit integers.
__host__ __device__ inline uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}
__host__ __device__ inline uint32_t lowbias32_inv(uint32_t x) {
  x ^= x >> 16;
  x *= 0x43021123U;  // inverse of 0x846ca68b modulo 2^32
  x ^= (x >> 15) ^ (x >> 30);
  x *= 0x1d69e2a5U;  // inverse of 0x7feb352d modulo 2^32
  x ^= x >> 16;
  return x;
}

// Shell ranking key of Eq. 11's batch: key(j) = lowbias32(lowbias32(id_j ^ a) ^ b)
// with (a, b) = low/high halves of stream_out(stream_out(seed ^ tag, eval), id_i).
struct ShellKey {
  uint32_t a, b;
};
__host__ __device__ inline uint64_t shell_eval_key(uint64_t seed, uint64_t eval) {
  return stream_out(seed ^ kTagShell, eval);
}
__host__ __device__ inline ShellKey shell_key_of(uint64_t eval_key, int32_t id_i) {
  uint64_t h = stream_out(eval_key, (uint64_t)(uint32_t)id_i);
  return ShellKey{(uint32_t)h, (uint32_t)(h >> 32)};
}
__host__ __device__ inline uint32_t shell_rank(ShellKey k, int32_t id_j) {
  return lowbias32(lowbias32((uint32_t)id_j ^ k.a) ^ k.b);
}
__host__ __device__ inline int32_t shell_id_of(ShellKey k, uint32_t rank) {
  return (int32_t)(lowbias32_inv(lowbias32_inv(rank) ^ k.b) ^ k.a);
}

// ---------------------------------------------------------------------------
// Geometry
// ---------------------------------------------------------------------------
struct Grid {
  int nx, ny, nz;     // cells per axis
  int ncell;          // nx * ny * nz (keys run over 2 * ncell: charged, then neutral)
  double L[3];        // box
  double inv_h[3];    // n_d / L_d (cell scale used by the binning key)
  // ghost shell (ghost_width > 0): the padded grid extends the native grid by
  // goff[d] cells on both sides; cell c of the native grid is padded cell
  // c + goff[d]. Zero layers without a ghost shell.
  int goff[3];
  int pnx, pny, pnz;  // padded cells per axis
  int pncell;         // pnx * pny * pnz
  double ghost_width;
};

// Wrap into [0, L): w = x - L floor(x / L); values pushed to L or below 0 by
// rounding map to 0. Written without contraction so every caller gets the
// same bits.
__host__ __device__ inline double wrap_coord(double x, double L) {
#pragma clang fp contract(off)
  double w = x - L * floor(x / L);
  if (w < 0.0 || w >= L) w = 0.0;
  return w;
}

// Cell index of a wrapped coordinate: min(n - 1, floor(w * inv_h)). Written
// so that a NaN (a failed step) lands in cell 0 instead of an undefined
// conversion: every cell index stays inside the grid.
__host__ __device__ inline int cell_coord(double w, double inv_h, int n) {
  const double t = w * inv_h;
  if (t >= 0.0 && t < (double)n) {
    const int c = (int)t;
    return c >= n ? n - 1 : c;
  }
  return t >= (double)n ? n - 1 : 0;
}

// floor(a / n) for the small offsets of a stencil (|a| within a few n): a
// compare-and-step loop instead of an integer division.
__host__ __device__ inline int floor_div(int a, int n) {
  int q = 0;
  while (a < 0) {
    a += n;
    --q;
  }
  while (a >= n) {
    a -= n;
    ++q;
  }
  return q;
}

// ---------------------------------------------------------------------------
// XCD-aware workgroup order
// ---------------------------------------------------------------------------
// The dispatcher hands workgroups to the 8 XCDs round-robin (workgroup b runs
// on XCD b mod 8), and each XCD has its own L2. xcd_block maps b to a
// logical index under which every XCD's workgroups are consecutive, so each
// L2 serves one contiguous range of the cell-ordered particles (a compact
// region of the box and its stencil neighbourhood) instead of all of it.
// A bijection of [0, nb) for any nb.
constexpr int kNumXcd = 8;
__host__ __device__ inline int64_t xcd_block(int64_t b, int64_t nb) {
  const int64_t x = b % kNumXcd, local = b / kNumXcd;
  const int64_t base = nb / kNumXcd, rem = nb % kNumXcd;
  return x * base + (x < rem ? x : rem) + local;
}

// ---------------------------------------------------------------------------
// Binning helpers (counting sort by cell key)
// ---------------------------------------------------------------------------
// Slot of this lane's particle in its key's bucket, one atomic per run of
// equal keys in consecutive lanes (all lanes of the wave call it; lanes with
// active = false take no slot and must carry a key no other lane has).
__device__ inline int run_slot(int k, bool active, int32_t *count) {
  const int lane = threadIdx.x & 63;
  const int kp = __shfl_up(k, 1, 64);
  const bool start = lane == 0 || kp != k;
  const unsigned long long starts = __ballot(start);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int leader = 63 - __clzll((long long)(starts & upto));
  const unsigned long long after = starts & ~upto;
  const int next = after ? __ffsll((long long)after) - 1 : 64;
  int base = 0;
  if (start && active) base = atomicAdd(&count[k], next - lane);
  base = __shfl(base, leader, 64);
  return base + (lane - leader);
}

// One thread per bucket: copy its entries to perm, checking the order, and
// sort them by insertion if they are out of order (entries are distinct).
__device__ inline void place_bucket(int lo, int hi, const int32_t *__restrict__ tmp, int32_t *__restrict__ perm) {
  bool sorted = true;
  int32_t prev = -1;
  for (int t = lo; t < hi; ++t) {
    const int32_t v = tmp[t];
    perm[t] = v;
    sorted = sorted && v > prev;
    prev = v;
  }
  if (sorted) return;
  for (int t = lo + 1; t < hi; ++t) {
    const int32_t v = perm[t];
    int u = t;
    while (u > lo && perm[u - 1] > v) {
      perm[u] = perm[u - 1];
      --u;
    }
    perm[u] = v;
  }
}

// ---------------------------------------------------------------------------
// Mode tables for the sampler (host-built, copied to the device)
// ---------------------------------------------------------------------------
struct ModeTable {
  int M[3];        // |m_d| <= M[d]
  int off[3];      // offset of axis d in the cdf array
  double S;        // normalizer of Eq. 9
  double V;        // box volume
  double L[3];
  int total;       // total cdf entries
  int kdist;       // rbe_kdist of the sample
  double kmin2;    // min_d (2 pi / L_d)^2: the smallest nonzero k^2 (RBE_KDIST_GAUSS_OVER_K2)
  double S2;       // sum_{k != 0} exp(-k^2/(4 alpha)) / k^2 over the table (RBE_KDIST_GAUSS_OVER_K2)
};

int axis_cutoff(double L, double alpha);
// Builds the per-axis cumulative tables (host). cdf must hold table.total
// entries; with cdf given and kdist = RBE_KDIST_GAUSS_OVER_K2 also the
// normalizer S2 (a sum over the whole table's lattice).
void build_mode_table(const double L[3], double alpha, ModeTable *t, double *cdf, int kdist = 0);
// Host sampler: draws P modes for (seed, eval).
int sample_modes_host(const ModeTable &t, const double *cdf, uint64_t seed, uint64_t eval, int P, int32_t *m,
                      double *w);
// Device sampler launch (cdf is a device copy of the host table).
// nev consecutive evaluations from eval (sample y at m + 3P y, w + P y, and
// the mode vectors as doubles at mkd + 3P y when mkd is given).
void launch_sample_modes(const ModeTable &t, const double *cdf_dev, uint64_t seed, uint64_t eval, int P,
                         int32_t *m, double *w, int *err_flag, hipStream_t st, int nev = 1, double *mkd = nullptr);

// ---------------------------------------------------------------------------
// Error flag bits (device int)
// ---------------------------------------------------------------------------
enum : int { kErrNonFinite = 1, kErrBadId = 2, kErrSampler = 4, kErrGhostOverflow = 8, kErrBarrier = 16,
             kErrNonNeutral = 32, kErrTileOverflow = 64 };

}  // namespace rbe
