// Fourier part of the RBE force (Sec. 2.1, Eq. 5, 7, 9; Sec. 2.3.1):
// structure factors rho(k_l) = sum_j q_j exp(i k_l . r_j) over the charged
// particles, then F_i = -kc q_i sum_l w_l k_l Im(exp(-i k_l . r_i) rho_l)
// (kc the Coulomb prefactor, 1 in reduced units).
//
// Phase: k_l . r_j = 2 pi t with t = m_l . s_j (s = r/L, the fractional
// coordinate). Whole turns are removed in FP64 (t - rint(t), exact for the
// fraction) before the sine and cosine, so the trigonometric argument is a
// fraction of a turn in [-1/2, 1/2] whatever the box size.
//
// Structure factor: thread = mode, particles walked in a wave-uniform loop
// (scalar loads of the packed (s, q) records), one partial sum per particle
// chunk and mode. A wave left with fewer than 64 modes (P not a multiple of
// 64) spreads each mode over several lanes that split the chunk's particles
// and adds their sums with a fixed butterfly. The chunk partials are summed
// in FP64 in a fixed order by a second kernel.
//
// Gather: thread = particle, modes walked in a wave-uniform loop with the
// per-mode coefficients (m, w Im rho, w Re rho) in scalar registers.
//
// FP32C form: the turn reduction stays FP64; the hardware turn-argument
// sine/cosine (v_sin_f32 / v_cos_f32 compute sin(2 pi x), cos(2 pi x)) run on
// the FP32 fraction; sums are FP32: blocks of 8 terms summed plainly, the
// block sums added with Kahan compensation.
#include "fourier_device.h"

namespace rbe {

constexpr int kModesPerBlock = 256;
// Terms summed in plain FP32 before their sum joins the Kahan-compensated
// total (FP32C kernels).
constexpr int kSumBlock = 8;

void fill_turn_table(double2 *host, int n) {
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int k = 0; k < n; ++k) {
    const long double a = two_pi * (long double)k / (long double)n;
    host[k] = make_double2((double)sinl(a), (double)cosl(a));
  }
}

__global__ void k_modes_to_double(int P, const int32_t *__restrict__ m, double *__restrict__ mkd) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < 3 * P) mkd[l] = (double)m[l];
}

void launch_modes_to_double(int P, const int32_t *m, double *mkd, hipStream_t st) {
  k_modes_to_double<<<(3 * P + 255) / 256, 256, 0, st>>>(P, m, mkd);
}

// ---------------------------------------------------------------------------
// structure factor partial sums
// ---------------------------------------------------------------------------
// A wave holds 64 consecutive modes. The last wave of a mode set whose size
// is not a multiple of 64 holds a < 64: its lanes then split as rep lanes per
// mode (rep the largest power of two with rep a <= 64), each taking every
// rep-th particle of the chunk, and the rep partial sums of a mode are added
// by a fixed butterfly, so that wave does 1/rep of the trips instead of all.
__device__ inline int wave_rep(int a) {
  int rep = 1;
  while (2 * rep * a <= 64) rep *= 2;
  return rep;
}

__global__ void __launch_bounds__(kModesPerBlock) k_rho_partial_f64(const int32_t *__restrict__ nq_ptr, int P,
                                                                     int nchunk_max,
                                                                     const double4 *__restrict__ sq,
                                                                     const double *__restrict__ mkd,
                                                                     const double2 *__restrict__ turn_tab,
                                                                     double2 *__restrict__ part) {
  static_assert(kModesPerBlock == kTurnTable, "one table entry per thread");
  __shared__ double2 tab[kTurnTable];
  __shared__ double4 rec[kModesPerBlock];  // the chunk's records, staged a round at a time
  const int64_t nq = *nq_ptr;
  int nchunks;
  const int chunk = rho_layout(nq, P, nchunk_max, &nchunks);
  if ((int)blockIdx.x >= nchunks) return;  // uniform over the block
  tab[threadIdx.x] = turn_tab[threadIdx.x];
  const int lane = threadIdx.x & 63;
  const int l0 = blockIdx.y * kModesPerBlock + (threadIdx.x & ~63);  // first mode of this wave
  const int a = max(0, min(64, P - l0));  // modes of this wave (0: it only stages records)
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = min(nq, j0 + chunk);
  // a == 64: one mode per lane; fewer: rep lanes per mode, each taking every
  // rep-th record, added by a fixed butterfly
  const int rep = a == 64 ? 1 : (a > 0 ? wave_rep(a) : 64);
  const int mi = lane / rep, ph = lane % rep;
  const bool active = mi < a;
  const int l = l0 + (active ? mi : 0);
  double mx = 0.0, my = 0.0, mz = 0.0;
  if (a > 0) {
    mx = mkd[l];
    my = mkd[P + l];
    mz = mkd[2 * P + l];
  }
  double re = 0.0, im = 0.0;
  for (int64_t b = j0; b < j1; b += kModesPerBlock) {
    const int cnt = (int)min((int64_t)kModesPerBlock, j1 - b);
    __syncthreads();  // the table is written; the previous round is no longer read
    if ((int)threadIdx.x < cnt) rec[threadIdx.x] = sq[b + threadIdx.x];
    __syncthreads();
    if (a == 0) continue;
#pragma unroll 4
    for (int u = ph; u < cnt; u += rep) {
      const double4 r = rec[u];
      const double t = turn_fraction(mx, my, mz, r.x, r.y, r.z);
      double sn, cs;
      sincos_turn_tab_f64(t, tab, &sn, &cs);
      re = fma(r.w, cs, re);
      im = fma(r.w, sn, im);
    }
  }
  if (a == 0) return;
  for (int o = rep >> 1; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  if (active && ph == 0) part[(int64_t)blockIdx.x * P + l] = make_double2(re, im);
}

// Record: x, y, z as doubles, the FP32 charge in the low word of w.
__device__ inline float rec_q(const double4 &r) { return __int_as_float(__double2loint(r.w)); }

__global__ void __launch_bounds__(kModesPerBlock) k_rho_partial_f32c(const int32_t *__restrict__ nq_ptr, int P,
                                                                      int nchunk_max,
                                                                      const double4 *__restrict__ sq,
                                                                      const double *__restrict__ mkd,
                                                                      double2 *__restrict__ part) {
  __shared__ double4 rec[kModesPerBlock];
  const int64_t nq = *nq_ptr;
  int nchunks;
  const int chunk = rho_layout(nq, P, nchunk_max, &nchunks);
  if ((int)blockIdx.x >= nchunks) return;  // uniform over the block
  const int lane = threadIdx.x & 63;
  const int l0 = blockIdx.y * kModesPerBlock + (threadIdx.x & ~63);
  // a wave past the last mode still stages records for the others
  const int a = max(0, min(64, P - l0));
  const int64_t j0 = (int64_t)blockIdx.x * chunk;
  const int64_t j1 = min(nq, j0 + chunk);
  const int rep = a == 64 ? 1 : (a > 0 ? wave_rep(a) : 64);
  const int mi = lane / rep, ph = lane % rep;
  const bool active = mi < a;
  const int l = l0 + (active ? mi : 0);
  double mx = 0.0, my = 0.0, mz = 0.0;
  if (a > 0) {
    mx = mkd[l];
    my = mkd[P + l];
    mz = mkd[2 * P + l];
  }
  float re = 0.f, re_c = 0.f, im = 0.f, im_c = 0.f;
  auto term = [&](const double4 &r, float &br, float &bi) {
    const float t = turn_f32(mx, my, mz, r.x, r.y, r.z);
    const float q = rec_q(r);
    br = fmaf(q, __builtin_amdgcn_cosf(t), br);
    bi = fmaf(q, __builtin_amdgcn_sinf(t), bi);
  };
  for (int64_t b = j0; b < j1; b += kModesPerBlock) {
    const int cnt = (int)min((int64_t)kModesPerBlock, j1 - b);
    __syncthreads();  // the previous round's records are no longer read
    if ((int)threadIdx.x < cnt) {
      const double4 s = sq[b + threadIdx.x];
      rec[threadIdx.x] = make_double4(s.x, s.y, s.z, __hiloint2double(0, __float_as_int((float)s.w)));
    }
    __syncthreads();
    if (a == 0) continue;
    if (rep == 1) {
      // blocks of kSumBlock terms summed in FP32, each block sum added to
      // the chunk's sum with Kahan compensation
      int u = 0;
      for (; u + kSumBlock <= cnt; u += kSumBlock) {
        double4 r[kSumBlock];  // all loads issued before the arithmetic
#pragma unroll
        for (int v = 0; v < kSumBlock; ++v) r[v] = rec[u + v];
        float br = 0.f, bi = 0.f;
#pragma unroll
        for (int v = 0; v < kSumBlock; ++v) term(r[v], br, bi);
        kahan_add(re, re_c, br);
        kahan_add(im, im_c, bi);
      }
      float br = 0.f, bi = 0.f;
      for (; u < cnt; ++u) term(rec[u], br, bi);
      kahan_add(re, re_c, br);
      kahan_add(im, im_c, bi);
    } else {
      for (int u = ph; u < cnt; u += rep) {
        const double4 r = rec[u];
        const float t = turn_f32(mx, my, mz, r.x, r.y, r.z);
        kahan_fma(re, re_c, rec_q(r), __builtin_amdgcn_cosf(t));
        kahan_fma(im, im_c, rec_q(r), __builtin_amdgcn_sinf(t));
      }
    }
  }
  if (a == 0) return;
  double dre = (double)re - (double)re_c, dim = (double)im - (double)im_c;
  for (int o = rep >> 1; o > 0; o >>= 1) {
    dre += __shfl_xor(dre, o, 64);
    dim += __shfl_xor(dim, o, 64);
  }
  if (active && ph == 0) part[(int64_t)blockIdx.x * P + l] = make_double2(dre, dim);
}

// rho_l = sum over chunks (fixed order: thread-strided FP64 sums, a fixed
// butterfly in each wave, then the waves in index order). Also forms the
// gather coefficients of each mode.
constexpr int kRhoFinalThreads = 256;
__global__ void __launch_bounds__(kRhoFinalThreads) k_rho_final(const int32_t *__restrict__ nq_ptr, int nchunk_max, int P,
                                                                const double2 *__restrict__ part,
                                                                const double *__restrict__ mkd,
                                                                const double *__restrict__ w, double kc,
                                                                double *__restrict__ rho,
                                                                GatherMode *__restrict__ modes,
                                                                double *__restrict__ rho_out) {
  __shared__ double2 wsum[kRhoFinalThreads / 64];
  int nchunks;
  (void)rho_layout(*nq_ptr, P, nchunk_max, &nchunks);
  const int l = blockIdx.x;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  double re = 0.0, im = 0.0;
#pragma unroll 4
  for (int c = threadIdx.x; c < nchunks; c += kRhoFinalThreads) {
    const double2 v = part[(int64_t)c * P + l];
    re += v.x;
    im += v.y;
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    re += __shfl_xor(re, o, 64);
    im += __shfl_xor(im, o, 64);
  }
  if (lane == 0) wsum[wave] = make_double2(re, im);
  __syncthreads();
  if (threadIdx.x == 0) {
    re = 0.0;
    im = 0.0;
    for (int k = 0; k < kRhoFinalThreads / 64; ++k) {
      re += wsum[k].x;
      im += wsum[k].y;
    }
    rho[l] = re;
    rho[P + l] = im;
    if (rho_out) {
      rho_out[l] = re;
      rho_out[P + l] = im;
    }
    GatherMode gm;
    gm.mx = mkd[l];
    gm.my = mkd[P + l];
    gm.mz = mkd[2 * P + l];
    const double wl = kc * w[l];
    gm.a = wl * im;
    gm.b = wl * re;
    gather_floats(gm);
    modes[l] = gm;
  }
}

void launch_rho_partial(int prec, const int32_t *nq, int64_t nq_max, int P, const double4 *sq,
                        const FourierBuffers &fb, hipStream_t st) {
  const int nchunks = rho_max_chunks(nq_max, P, fb.nchunk_max);
  dim3 grid((unsigned)nchunks, (unsigned)((P + kModesPerBlock - 1) / kModesPerBlock));
  if (prec == RBE_FP32C)
    k_rho_partial_f32c<<<grid, kModesPerBlock, 0, st>>>(nq, P, fb.nchunk_max, sq, fb.mkd, fb.part);
  else
    k_rho_partial_f64<<<grid, kModesPerBlock, 0, st>>>(nq, P, fb.nchunk_max, sq, fb.mkd, fb.turn_tab, fb.part);
}

void launch_rho_final(const int32_t *nq, int P, const FourierBuffers &fb, const double *w, double kc,
                      double *rho_out, hipStream_t st) {
  k_rho_final<<<P, kRhoFinalThreads, 0, st>>>(nq, fb.nchunk_max, P, fb.part, fb.mkd, w, kc, fb.rho, fb.modes,
                                              rho_out);
}

// ---------------------------------------------------------------------------
// force gather (adds F^F into f for the charged range)
// ---------------------------------------------------------------------------
// Mode groups: blockIdx.y = g sums the modes [g M, min(P, (g + 1) M)); with
// one group the force is applied here, with several the group's sums go to
// gpart[g * stride + i] and k_gather_reduce adds the groups in order.
__global__ void __launch_bounds__(kTurnTable) k_gather_f64(const int32_t *__restrict__ nq_ptr, int P, int M,
                                                           const double4 *__restrict__ sq,
                                                           const GatherMode *__restrict__ modes,
                                                           const double2 *__restrict__ turn_tab, double kx,
                                                           double ky, double kz, double *__restrict__ fx,
                                                           double *__restrict__ fy, double *__restrict__ fz,
                                                           double4 *__restrict__ gpart, int64_t stride) {
  __shared__ double2 tab[kTurnTable];
  const int64_t nq = *nq_ptr;
  if ((int64_t)blockIdx.x * blockDim.x >= nq) return;  // uniform over the block
  tab[threadIdx.x] = turn_tab[threadIdx.x];
  __syncthreads();
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nq) return;
  const double4 s = sq[i];
  double gx = 0.0, gy = 0.0, gz = 0.0;
  const int lb = blockIdx.y * M, le = min(P, lb + M);
#pragma unroll 4
  for (int l = lb; l < le; ++l) {
    const GatherMode gm = modes[l];
    const double t = turn_fraction(gm.mx, gm.my, gm.mz, s.x, s.y, s.z);
    double sn, cs;
    sincos_turn_tab_f64(t, tab, &sn, &cs);
    const double g = gm.a * cs - gm.b * sn;  // w Im(exp(-i theta) rho)
    gx = fma(g, gm.mx, gx);
    gy = fma(g, gm.my, gy);
    gz = fma(g, gm.mz, gz);
  }
  if (gpart) {
    gpart[blockIdx.y * stride + i] = make_double4(gx, gy, gz, 0.0);
    return;
  }
  const double q = s.w;
  fx[i] -= q * kx * gx;
  fy[i] -= q * ky * gy;
  fz[i] -= q * kz * gz;
}

// Two charged particles per thread (i and i + 256 of the block's 512); every
// lane reads the same mode at a time (wave-uniform scalar loads, which
// deliver a record once per wave), and each mode read serves both particles.
// Staging the modes in LDS instead measured slower: the broadcast LDS reads
// cost more than the load latency they hide.
constexpr int kGatherThreads = 256;
constexpr int kGatherPerBlock = 2 * kGatherThreads;
__global__ void __launch_bounds__(kGatherThreads) k_gather_f32c(const int32_t *__restrict__ nq_ptr, int P, int M,
                                                                const double4 *__restrict__ sq,
                                                                const GatherMode *__restrict__ modes, double kx,
                                                                double ky, double kz, double *__restrict__ fx,
                                                                double *__restrict__ fy, double *__restrict__ fz,
                                                                double4 *__restrict__ gpart, int64_t stride) {
  const int64_t nq = *nq_ptr;
  const int64_t i = blockIdx.x * (int64_t)kGatherPerBlock + threadIdx.x, i2 = i + kGatherThreads;
  if (i >= nq) return;
  const bool two = i2 < nq;
  const double4 s = sq[i], s2 = two ? sq[i2] : s;
  float gx = 0.f, gy = 0.f, gz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
  float hx = 0.f, hy = 0.f, hz = 0.f, dx = 0.f, dy = 0.f, dz = 0.f;
  auto term = [&](int l, float &bx, float &by, float &bz, float &ex, float &ey, float &ez) {
    const GatherMode gm = modes[l];
    const float t = turn_f32(gm.mx, gm.my, gm.mz, s.x, s.y, s.z);
    const float t2 = turn_f32(gm.mx, gm.my, gm.mz, s2.x, s2.y, s2.z);
    const float g = fmaf(gm.af, __builtin_amdgcn_cosf(t), -gm.bf * __builtin_amdgcn_sinf(t));
    const float g2 = fmaf(gm.af, __builtin_amdgcn_cosf(t2), -gm.bf * __builtin_amdgcn_sinf(t2));
    bx = fmaf(g, gm.mxf, bx);
    by = fmaf(g, gm.myf, by);
    bz = fmaf(g, gm.mzf, bz);
    ex = fmaf(g2, gm.mxf, ex);
    ey = fmaf(g2, gm.myf, ey);
    ez = fmaf(g2, gm.mzf, ez);
  };
  // blocks of kSumBlock modes summed in FP32, each block sum added with
  // Kahan compensation (a group's first mode is a multiple of kSumBlock, so
  // the blocks run over the modes in order and only the last one is short)
  const int lb = blockIdx.y * M, le = min(P, lb + M);
  int l = lb;
  for (; l + kSumBlock <= le; l += kSumBlock) {
    float bx = 0.f, by = 0.f, bz = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
#pragma unroll
    for (int u = 0; u < kSumBlock; ++u) term(l + u, bx, by, bz, ex, ey, ez);
    kahan_add(gx, cx, bx);
    kahan_add(gy, cy, by);
    kahan_add(gz, cz, bz);
    kahan_add(hx, dx, ex);
    kahan_add(hy, dy, ey);
    kahan_add(hz, dz, ez);
  }
  {
    float bx = 0.f, by = 0.f, bz = 0.f, ex = 0.f, ey = 0.f, ez = 0.f;
    for (; l < le; ++l) term(l, bx, by, bz, ex, ey, ez);
    kahan_add(gx, cx, bx);
    kahan_add(gy, cy, by);
    kahan_add(gz, cz, bz);
    kahan_add(hx, dx, ex);
    kahan_add(hy, dy, ey);
    kahan_add(hz, dz, ez);
  }
  auto put = [&](int64_t k, const double4 &sk, float ax, float acx, float ay, float acy, float az, float acz) {
    const double sx = (double)ax - (double)acx, sy = (double)ay - (double)acy, sz = (double)az - (double)acz;
    if (gpart) {
      gpart[blockIdx.y * stride + k] = make_double4(sx, sy, sz, 0.0);
      return;
    }
    const double q = sk.w;
    fx[k] -= q * kx * sx;
    fy[k] -= q * ky * sy;
    fz[k] -= q * kz * sz;
  };
  put(i, s, gx, cx, gy, cy, gz, cz);
  if (two) put(i2, s2, hx, dx, hy, dy, hz, dz);
}

// The groups' sums of each charged particle added in group order (FP64),
// then applied like the single-group gather.
__global__ void __launch_bounds__(256) k_gather_reduce(const int32_t *__restrict__ nq_ptr, int G, int64_t stride,
                                                       const double4 *__restrict__ gpart,
                                                       const double4 *__restrict__ sq, double kx, double ky,
                                                       double kz, double *__restrict__ fx, double *__restrict__ fy,
                                                       double *__restrict__ fz) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= *nq_ptr) return;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int g = 0; g < G; ++g) {
    const double4 v = gpart[g * stride + i];
    gx += v.x;
    gy += v.y;
    gz += v.z;
  }
  const double q = sq[i].w;
  fx[i] -= q * kx * gx;
  fy[i] -= q * ky * gy;
  fz[i] -= q * kz * gz;
}

// Mode groups of the gather: one unless the charged range alone gives too few
// blocks to fill the GPU (a small system with many modes, such as the full
// Ewald lattice), then enough groups of M modes (a multiple of the staging
// round) for about 1024 blocks, within the partial-sum buffer.
static int gather_split(int64_t nq_max, int P, const FourierBuffers &fb, int *M) {
  const int64_t pb = (nq_max + 255) / 256;
  *M = P;
  if (!fb.gpart || pb >= 512 || P < 4 * kGatherThreads) return 1;
  int64_t G = (1024 + pb - 1) / pb;
  while (G > 1 && G * pb * 256 > kGatherPartMax) --G;
  const int64_t m = ((P + G - 1) / G + kGatherThreads - 1) / kGatherThreads * kGatherThreads;
  *M = (int)m;
  return (int)((P + m - 1) / m);
}

void launch_fourier_gather(int prec, const int32_t *nq, int64_t nq_max, int P, const double4 *sq,
                           const FourierBuffers &fb, const Grid &g, double *fx, double *fy, double *fz,
                           hipStream_t st) {
  if (nq_max <= 0) return;
  const unsigned blocks = (unsigned)((nq_max + 255) / 256);
  const double kx = kTwoPi / g.L[0], ky = kTwoPi / g.L[1], kz = kTwoPi / g.L[2];
  int M;
  const int G = gather_split(nq_max, P, fb, &M);
  double4 *gp = G > 1 ? fb.gpart : nullptr;
  const int64_t stride = (int64_t)blocks * 256;
  const dim3 grid(blocks, (unsigned)G);
  if (prec == RBE_FP32C)
    k_gather_f32c<<<dim3((unsigned)((nq_max + kGatherPerBlock - 1) / kGatherPerBlock), (unsigned)G), kGatherThreads,
                    0, st>>>(nq, P, M, sq, fb.modes, kx, ky, kz, fx, fy, fz, gp, stride);
  else
    k_gather_f64<<<grid, kTurnTable, 0, st>>>(nq, P, M, sq, fb.modes, fb.turn_tab, kx, ky, kz, fx, fy, fz, gp,
                                              stride);
  if (G > 1) k_gather_reduce<<<blocks, 256, 0, st>>>(nq, G, stride, gp, sq, kx, ky, kz, fx, fy, fz);
}

}  // namespace rbe
