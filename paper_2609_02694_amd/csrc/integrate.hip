// Data movement, reductions and the velocity-Verlet kernels (all bound by
// HBM bandwidth): packed sorted copies, the inverse id map, force scatter,
// the fixed-order mean of Eq. 12, and the half-kick / drift / wrap steps.
#include "kernels.h"

namespace rbe {

__global__ void __launch_bounds__(256) k_gather_sorted(int64_t n, const int32_t *__restrict__ perm,
                                                       const double *__restrict__ x, const double *__restrict__ y,
                                                       const double *__restrict__ z, const double *__restrict__ q,
                                                       const int32_t *__restrict__ id, Grid g,
                                                       double4 *__restrict__ xq, double4 *__restrict__ sq,
                                                       int32_t *__restrict__ ids) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int j = perm[k];
  const double wx = wrap_coord(x[j], g.L[0]), wy = wrap_coord(y[j], g.L[1]), wz = wrap_coord(z[j], g.L[2]);
  const double qq = q[j];
  xq[k] = make_double4(wx, wy, wz, qq);
  if (qq != 0.0) sq[k] = make_double4(wx / g.L[0], wy / g.L[1], wz / g.L[2], qq);
  if (id) ids[k] = id[j];
}

void launch_gather_sorted(int64_t n, const int32_t *perm, const double *x, const double *y, const double *z,
                          const double *q, const int32_t *id, const Grid &g, Sorted s, hipStream_t st) {
  if (n <= 0) return;
  k_gather_sorted<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, perm, x, y, z, q, id, g, s.xq, s.sq, s.id);
}

// inv must hold -1 everywhere on entry. Ids outside [0, n) and repeated ids
// are flagged; the near-field kernel skips any batch member whose id does not
// map back to a slot in [0, n).
__global__ void k_inverse_ids(int64_t n, const int32_t *__restrict__ id, int32_t *__restrict__ inv, int *err) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int32_t v = id[k];
  if (v < 0 || (int64_t)v >= n) {
    atomicOr(err, kErrBadId);
    return;
  }
  if (atomicCAS(&inv[v], -1, (int32_t)k) != -1) atomicOr(err, kErrBadId);
}

void launch_inverse_ids(int64_t n, const int32_t *id_sorted, int32_t *inv, int *err, hipStream_t st) {
  if (n <= 0) return;
  launch_fill_i32(inv, n, -1, st);
  k_inverse_ids<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, id_sorted, inv, err);
}

__global__ void k_scatter_forces(int64_t n, const int32_t *__restrict__ perm, const double *__restrict__ fx,
                                 const double *__restrict__ fy, const double *__restrict__ fz, double *__restrict__ ox,
                                 double *__restrict__ oy, double *__restrict__ oz) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int j = perm[k];
  ox[j] = fx[k];
  oy[j] = fy[k];
  oz[j] = fz[k];
}

void launch_scatter_forces(int64_t n, const int32_t *perm, const double *fx, const double *fy, const double *fz,
                           double *ox, double *oy, double *oz, hipStream_t st) {
  if (n <= 0) return;
  k_scatter_forces<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, perm, fx, fy, fz, ox, oy, oz);
}

// ---------------------------------------------------------------------------
// fixed-order mean (Eq. 12)
// ---------------------------------------------------------------------------
constexpr int kMeanThreads = 256;
constexpr int64_t kMeanPerBlock = 2048;

int mean_blocks(int64_t n) { return (int)((n + kMeanPerBlock - 1) / kMeanPerBlock); }

__device__ inline double block_sum_fixed(double v, double *lds) {
  // fixed butterfly inside each wave, then waves in index order
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kMeanThreads / 64; ++w) s += lds[w];
  __syncthreads();
  return s;
}

__global__ void __launch_bounds__(kMeanThreads) k_mean_partial(int64_t n, const double *__restrict__ fx,
                                                               const double *__restrict__ fy,
                                                               const double *__restrict__ fz,
                                                               double *__restrict__ partials) {
  __shared__ double lds[kMeanThreads / 64];
  const int64_t b0 = (int64_t)blockIdx.x * kMeanPerBlock;
  const int64_t b1 = min(n, b0 + kMeanPerBlock);
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int64_t i = b0 + threadIdx.x; i < b1; i += kMeanThreads) {
    s0 += fx[i];
    s1 += fy[i];
    s2 += fz[i];
  }
  s0 = block_sum_fixed(s0, lds);
  s1 = block_sum_fixed(s1, lds);
  s2 = block_sum_fixed(s2, lds);
  if (threadIdx.x == 0) {
    partials[3 * blockIdx.x] = s0;
    partials[3 * blockIdx.x + 1] = s1;
    partials[3 * blockIdx.x + 2] = s2;
  }
}

__global__ void __launch_bounds__(kMeanThreads) k_mean_final(int nblk, int64_t n, const double *__restrict__ partials,
                                                             double *__restrict__ mean) {
  __shared__ double lds[kMeanThreads / 64];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll 4
  for (int b = threadIdx.x; b < nblk; b += kMeanThreads) {
    s0 += partials[3 * b];
    s1 += partials[3 * b + 1];
    s2 += partials[3 * b + 2];
  }
  s0 = block_sum_fixed(s0, lds);
  s1 = block_sum_fixed(s1, lds);
  s2 = block_sum_fixed(s2, lds);
  if (threadIdx.x == 0) {
    const double inv = 1.0 / (double)n;
    mean[0] = s0 * inv;
    mean[1] = s1 * inv;
    mean[2] = s2 * inv;
  }
}

void launch_mean3(int64_t n, const double *fx, const double *fy, const double *fz, double *partials, double *mean,
                  hipStream_t st) {
  const int nb = mean_blocks(n);
  if (nb > 0) k_mean_partial<<<nb, kMeanThreads, 0, st>>>(n, fx, fy, fz, partials);
  k_mean_final<<<1, kMeanThreads, 0, st>>>(nb, n, partials, mean);
}

// ---------------------------------------------------------------------------
// velocity Verlet
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_kick(int64_t n, double h, const double *__restrict__ mean,
                                              double *__restrict__ fx, double *__restrict__ fy,
                                              double *__restrict__ fz, double *__restrict__ vx,
                                              double *__restrict__ vy, double *__restrict__ vz, int *err) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  double a = fx[i], b = fy[i], c = fz[i];
  if (mean) {
    a -= mean[0];
    b -= mean[1];
    c -= mean[2];
    fx[i] = a;
    fy[i] = b;
    fz[i] = c;
  }
  const double u = vx[i] + h * a, v = vy[i] + h * b, w = vz[i] + h * c;
  vx[i] = u;
  vy[i] = v;
  vz[i] = w;
  if (!isfinite(u) || !isfinite(v) || !isfinite(w)) atomicOr(err, kErrNonFinite);
}

void launch_kick(int64_t n, double h, const double *mean, double *fx, double *fy, double *fz, double *vx, double *vy,
                 double *vz, int *err, hipStream_t st) {
  if (n <= 0) return;
  k_kick<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, h, mean, fx, fy, fz, vx, vy, vz, err);
}

__global__ void __launch_bounds__(256) k_sub_mean(int64_t n, const double *__restrict__ mean, double *__restrict__ fx,
                                                  double *__restrict__ fy, double *__restrict__ fz) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  fx[i] -= mean[0];
  fy[i] -= mean[1];
  fz[i] -= mean[2];
}

void launch_sub_mean(int64_t n, const double *mean, double *fx, double *fy, double *fz, hipStream_t st) {
  if (n <= 0) return;
  k_sub_mean<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, mean, fx, fy, fz);
}

// v <- s v + h f (s = *scale when given: the thermostat's velocity scaling
// of the NVT step; the NVE step passes no scale); x <- wrap(x + dt v).
// Binning key of a drifted particle, computed from the stored (wrapped)
// position exactly as the keys pass of the counting sort computes it, and its
// run slot (every lane of the wave takes part; lanes past n carry a key no
// other lane has).
__device__ inline void drift_key(const BinKeyOut &bk, const Grid &g, int64_t i, bool active, double x, double y,
                                 double z) {
  int k = -1 - (int)(threadIdx.x & 63);
  if (active) {
    const int cx = cell_coord(wrap_coord(x, g.L[0]), g.inv_h[0], g.nx);
    const int cy = cell_coord(wrap_coord(y, g.L[1]), g.inv_h[1], g.ny);
    const int cz = cell_coord(wrap_coord(z, g.L[2]), g.inv_h[2], g.nz);
    k = (bk.q[i] == 0.0 ? g.ncell : 0) + (cz * g.ny + cy) * g.nx + cx;
    bk.key[i] = k;
  }
  const int sl = run_slot(k, active, bk.count);
  if (active) bk.slot[i] = sl;
}

__global__ void __launch_bounds__(256) k_kick_drift(int64_t n, double h, double dt, Grid g,
                                                    const double *__restrict__ scale,
                                                    const double *__restrict__ fx, const double *__restrict__ fy,
                                                    const double *__restrict__ fz, double *__restrict__ vx,
                                                    double *__restrict__ vy, double *__restrict__ vz,
                                                    double *__restrict__ x, double *__restrict__ y,
                                                    double *__restrict__ z, int *err, BinKeyOut bk) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = i < n;
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if (active) {
    double v0x = vx[i], v0y = vy[i], v0z = vz[i];
    if (scale) {
      const double sc = *scale;
      v0x *= sc;
      v0y *= sc;
      v0z *= sc;
    }
    const double u = v0x + h * fx[i], v = v0y + h * fy[i], w = v0z + h * fz[i];
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
    nx = wrap_coord(x[i] + dt * u, g.L[0]);
    ny = wrap_coord(y[i] + dt * v, g.L[1]);
    nz = wrap_coord(z[i] + dt * w, g.L[2]);
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    if (!isfinite(u) || !isfinite(v) || !isfinite(w)) atomicOr(err, kErrNonFinite);
  }
  if (bk.key) drift_key(bk, g, i, active, nx, ny, nz);
}

// The second half-kick of one step followed by the first half-kick and drift
// of the next (both half-kicks with the same force, mean-corrected when
// `mean` is given), in one pass: the same two roundings of v as the separate
// kernels, without writing the corrected force back (the next evaluation
// overwrites it).
__global__ void __launch_bounds__(256) k_kick_kick_drift(int64_t n, double h, double dt, Grid g,
                                                         const double *__restrict__ mean,
                                                         const double *__restrict__ fx,
                                                         const double *__restrict__ fy,
                                                         const double *__restrict__ fz, double *__restrict__ vx,
                                                         double *__restrict__ vy, double *__restrict__ vz,
                                                         double *__restrict__ x, double *__restrict__ y,
                                                         double *__restrict__ z, int *err, BinKeyOut bk) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const bool active = i < n;
  double nx = 0.0, ny = 0.0, nz = 0.0;
  if (active) {
    double a = fx[i], b = fy[i], c = fz[i];
    if (mean) {
      a -= mean[0];
      b -= mean[1];
      c -= mean[2];
    }
    const double u1 = vx[i] + h * a, v1 = vy[i] + h * b, w1 = vz[i] + h * c;
    const double u = u1 + h * a, v = v1 + h * b, w = w1 + h * c;
    vx[i] = u;
    vy[i] = v;
    vz[i] = w;
    nx = wrap_coord(x[i] + dt * u, g.L[0]);
    ny = wrap_coord(y[i] + dt * v, g.L[1]);
    nz = wrap_coord(z[i] + dt * w, g.L[2]);
    x[i] = nx;
    y[i] = ny;
    z[i] = nz;
    if (!isfinite(u1) || !isfinite(v1) || !isfinite(w1) || !isfinite(u) || !isfinite(v) || !isfinite(w))
      atomicOr(err, kErrNonFinite);
  }
  if (bk.key) drift_key(bk, g, i, active, nx, ny, nz);
}
void launch_kick_kick_drift(int64_t n, double h, double dt, const Grid &g, const double *mean, const double *fx,
                            const double *fy, const double *fz, double *vx, double *vy, double *vz, double *x,
                            double *y, double *z, int *err, BinKeyOut bk, hipStream_t st) {
  if (n <= 0) return;
  k_kick_kick_drift<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, h, dt, g, mean, fx, fy, fz, vx, vy, vz, x, y, z,
                                                                 err, bk);
}

void launch_kick_drift(int64_t n, double h, double dt, const Grid &g, const double *scale, const double *fx,
                       const double *fy, const double *fz, double *vx, double *vy, double *vz, double *x, double *y,
                       double *z, int *err, BinKeyOut bk, hipStream_t st) {
  if (n <= 0) return;
  k_kick_drift<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, h, dt, g, scale, fx, fy, fz, vx, vy, vz, x, y, z,
                                                            err, bk);
}

// ---------------------------------------------------------------------------
// Nose-Hoover thermostat (NVT)
// ---------------------------------------------------------------------------
// Grid-stride partial sums of |v|^2 (fixed block count, fixed order), with
// the second half-kick v += h (f - mean) applied first when h != 0 (the
// corrected force is written back, as k_kick does).
constexpr int kNhBlocks = 1024;
int nh_part_len() { return kNhBlocks; }

__global__ void __launch_bounds__(kMeanThreads) k_kick_vsq(int64_t n, double h, const double *__restrict__ mean,
                                                           double *__restrict__ fx, double *__restrict__ fy,
                                                           double *__restrict__ fz, double *__restrict__ vx,
                                                           double *__restrict__ vy, double *__restrict__ vz,
                                                           double *__restrict__ part, int *err) {
  __shared__ double lds[kMeanThreads / 64];
  double s = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kMeanThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kMeanThreads) {
    double u = vx[i], v = vy[i], w = vz[i];
    if (h != 0.0) {
      double a = fx[i], b = fy[i], c = fz[i];
      if (mean) {
        a -= mean[0];
        b -= mean[1];
        c -= mean[2];
        fx[i] = a;
        fy[i] = b;
        fz[i] = c;
      }
      u += h * a;
      v += h * b;
      w += h * c;
      vx[i] = u;
      vy[i] = v;
      vz[i] = w;
      if (!isfinite(u) || !isfinite(v) || !isfinite(w)) atomicOr(err, kErrNonFinite);
    }
    s += u * u + v * v + w * w;
  }
  s = block_sum_fixed(s, lds);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// One half-step of the thermostat on the kinetic energy K:
//   xi += (dt/4) G(K);  s = exp(-xi dt/2);  eta += xi dt/2;  K <- s^2 K;
//   xi += (dt/4) G(K),  G(K) = (2K - N_f kT)/Q.
__device__ inline double nh_half(const NhParams &q, double *K, double *xi, double *eta) {
  *xi += 0.25 * q.dt * ((2.0 * *K - q.nf * q.kT) / q.Q);
  const double s = exp(-0.5 * q.dt * *xi);
  *eta += 0.5 * q.dt * *xi;
  *K *= s * s;
  *xi += 0.25 * q.dt * ((2.0 * *K - q.nf * q.kT) / q.Q);
  return s;
}

// K = (m/2) sum |v|^2 from the partials; then the end half of one step
// (END) and/or the start half of the next (START). nh = {xi, eta} is
// advanced in place; *scale receives the product of the velocity scalings,
// applied by the next k_kick_drift (or k_scale_v after a call's last step).
__global__ void __launch_bounds__(kMeanThreads) k_nh_thermo(int nb, const double *__restrict__ part, NhParams q,
                                                            int mode, double *__restrict__ nh,
                                                            double *__restrict__ scale) {
  __shared__ double lds[kMeanThreads / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nb; b += kMeanThreads) s += part[b];
  s = block_sum_fixed(s, lds);
  if (threadIdx.x == 0) {
    double K = 0.5 * q.mass * s, xi = nh[0], eta = nh[1], sc = 1.0;
    if (mode & kNhEnd) sc *= nh_half(q, &K, &xi, &eta);
    if (mode & kNhStart) sc *= nh_half(q, &K, &xi, &eta);
    nh[0] = xi;
    nh[1] = eta;
    *scale = sc;
  }
}

__global__ void __launch_bounds__(256) k_scale_v(int64_t n, const double *__restrict__ scale, double *__restrict__ vx,
                                                 double *__restrict__ vy, double *__restrict__ vz) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sc = *scale;
  vx[i] *= sc;
  vy[i] *= sc;
  vz[i] *= sc;
}

void launch_nh(int64_t n, double h, const double *mean, double *fx, double *fy, double *fz, double *vx, double *vy,
               double *vz, const NhParams &q, int mode, double *part, double *nh, double *scale, int *err,
               hipStream_t st) {
  int64_t nb = (n + kMeanThreads - 1) / kMeanThreads;
  if (nb > kNhBlocks) nb = kNhBlocks;
  if (nb < 1) nb = 1;
  k_kick_vsq<<<(unsigned)nb, kMeanThreads, 0, st>>>(n, h, mean, fx, fy, fz, vx, vy, vz, part, err);
  k_nh_thermo<<<1, kMeanThreads, 0, st>>>((int)nb, part, q, mode, nh, scale);
}

void launch_scale_v(int64_t n, const double *scale, double *vx, double *vy, double *vz, hipStream_t st) {
  if (n <= 0) return;
  k_scale_v<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, scale, vx, vy, vz);
}

}  // namespace rbe
