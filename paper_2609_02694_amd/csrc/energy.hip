// Energy terms of the Ewald splitting (Sec. 2.1): the screened real-space
// Coulomb energy (Eq. 4) and the LJ energy (Eq. 2) over every pair inside
// the cutoffs, the importance-sampled Fourier energy of a mode sample
// (Eq. 5 with the sampling of Eq. 9), the self energy (Eq. 6), the kinetic
// energy, and the virials of the three potential terms (minus their
// derivatives under a uniform dilation of positions and box), from which
// the pressure follows. Diagnostics, so always FP64, with the device
// library's sqrt, division, exp and erfc rather than the force kernels'
// polynomials.
//
// Every sum has one fixed order: per-thread sums, a fixed butterfly in each
// wave, the waves of a block in index order, then the block partials in
// index order (thread-strided sums, butterfly, waves) in a one-block final
// kernel. Results are a pure function of the inputs and the grid.
#include "pair_device.h"

namespace rbe {

constexpr int kEnergyThreads = 256;
constexpr int kEnergySqBlocks = 1024;  // grid of the q^2 / v^2 sums

// Sum of v over the block; the result is valid in thread 0.
__device__ inline double block_sum(double v, double *lds) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();  // lds may still be read from a previous call
  if (lane == 0) lds[wave] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int k = 0; k < kEnergyThreads / 64; ++k) s += lds[k];
  return s;
}

// Near-field energy and virial of particle i (sorted order), halved so that
// the sum over i counts each pair once:
//   u_i = 1/2 sum_{j != i} [kc q_i q_j erfc(sqrt(a) r)/r   (r <= r_coul)
//                           + 4 eps ((sigma/r)^12 - (sigma/r)^6) (r <= r_lj)]
//   w_i = 1/2 sum_{j != i} d_ij . F_ij = 1/2 sum r^2 (kc q_i q_j G(r) + G_LJ(r)),
//         r^2 G = erfc(sqrt(a) r)/r + 2 sqrt(a/pi) exp(-a r^2),
//         r^2 G_LJ = 24 eps (2 (sigma/r)^12 - (sigma/r)^6)        (Eq. 8)
// over the minimum image. Species layout as in the force kernels: charged i
// (q_i != 0, the range [0, nq) of the cell order) walk the charged block out to max(r_coul, r_lj) and the neutral
// block out to r_lj; neutral i walk both blocks out to r_lj.
// part[4 b + 0..3] = Coulomb energy, LJ energy, Coulomb virial, LJ virial of
// block b.
__global__ void __launch_bounds__(kEnergyThreads) k_energy_near(PairParams pp, double lj4, double two_sqrt_a_pi,
                                                                int64_t n, const double4 *__restrict__ xq,
                                                                const int32_t *__restrict__ cell_start,
                                                                double *__restrict__ part) {
  __shared__ double lds[kEnergyThreads / 64];
  const int64_t i = blockIdx.x * (int64_t)kEnergyThreads + threadIdx.x;
  double uc = 0.0, ul = 0.0, wc = 0.0, wl = 0.0;
  if (i < n) {
    const Grid &g = pp.g;
    const double4 pi4 = xq[i];
    const double xi = pi4.x, yi = pi4.y, zi = pi4.z, qi = pi4.w;
    const int cx = cell_coord(xi, g.inv_h[0], g.nx);
    const int cy = cell_coord(yi, g.inv_h[1], g.ny);
    const int cz = cell_coord(zi, g.inv_h[2], g.nz);
    auto visit = [&](int j, const double4 &pj, int, double shx, double shy, double shz) {
      const double dx = (xi - pj.x) - shx, dy = (yi - pj.y) - shy, dz = (zi - pj.z) - shz;
      const double r2 = sq_dist(dx, dy, dz);
      if (r2 == 0.0 && j == (int)i) return;
      if (pp.do_coul && r2 <= pp.rc2 && qi != 0.0 && pj.w != 0.0) {
        const double r = sqrt(r2);
        const double qq = pp.kc * qi * pj.w;
        const double er = erfc(pp.sqrt_alpha * r) / r;
        uc += qq * er;
        wc += qq * (er + two_sqrt_a_pi * exp(-pp.alpha * r2));
      }
      if (pp.do_lj && r2 <= pp.rlj2) {
        const double s2 = pp.sig2 / r2, s6 = s2 * s2 * s2;
        ul += s6 * s6 - s6;
        wl += 2.0 * s6 * s6 - s6;
      }
    };
    const Reach rq{xi, yi, zi, pp.rq2}, rlj{xi, yi, zi, pp.rlj2};
    if (qi != 0.0) {
      for_stencil<false>(g, cell_start, xq, nullptr, 0, cx, cy, cz, pp.s_coul, rq, visit);
      if (pp.do_lj) for_stencil<false>(g, cell_start, xq, nullptr, 1, cx, cy, cz, pp.s_lj, rlj, visit);
    } else if (pp.do_lj) {
      for_stencil<false>(g, cell_start, xq, nullptr, 0, cx, cy, cz, pp.s_lj, rlj, visit);
      for_stencil<false>(g, cell_start, xq, nullptr, 1, cx, cy, cz, pp.s_lj, rlj, visit);
    }
    uc *= 0.5;
    ul *= 0.5 * lj4;
    wc *= 0.5;
    wl *= 0.5 * pp.eps24;
  }
  const double sc = block_sum(uc, lds);
  const double sl = block_sum(ul, lds);
  const double vc = block_sum(wc, lds);
  const double vl = block_sum(wl, lds);
  if (threadIdx.x == 0) {
    part[4 * blockIdx.x] = sc;
    part[4 * blockIdx.x + 1] = sl;
    part[4 * blockIdx.x + 2] = vc;
    part[4 * blockIdx.x + 3] = vl;
  }
}

// part[2 b] = sum q_i^2 and part[2 b + 1] = sum |v_i|^2 over the particles
// of block b's grid-stride sequence (caller order; v may be absent).
__global__ void __launch_bounds__(kEnergyThreads) k_energy_sq(int64_t n, const double *__restrict__ q,
                                                              const double *__restrict__ vx,
                                                              const double *__restrict__ vy,
                                                              const double *__restrict__ vz,
                                                              double *__restrict__ part) {
  __shared__ double lds[kEnergyThreads / 64];
  double sq = 0.0, sv = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)kEnergyThreads + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kEnergyThreads) {
    sq += q[i] * q[i];
    if (vx) sv += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
  }
  const double a = block_sum(sq, lds);
  const double b = block_sum(sv, lds);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = a;
    part[2 * blockIdx.x + 1] = b;
  }
}

// Thread-strided sum of part[stride * b + off] over b < nb (block_sum order).
__device__ inline double sum_partials(const double *part, int64_t nb, int stride, int off, double *lds) {
  double s = 0.0;
  for (int64_t b = threadIdx.x; b < nb; b += kEnergyThreads) s += part[stride * b + off];
  return block_sum(s, lds);
}

// One block: out[0] Coulomb real, out[1] LJ, out[2] Fourier, out[3] self,
// out[4] kinetic, out[5..7] virials of the Coulomb real, LJ and Fourier terms.
__global__ void __launch_bounds__(kEnergyThreads) k_energy_final(EnergyFinal a) {
  __shared__ double lds[kEnergyThreads / 64];
  double near[4] = {0.0, 0.0, 0.0, 0.0};
  if (a.near_part)
    for (int t = 0; t < 4; ++t) near[t] = sum_partials(a.near_part, a.nb_near, 4, t, lds);
  double uf = 0.0, wf = 0.0;
  if (a.rho) {
    // U^{F,*} = kc (1/2) sum_l w_l |rho_l|^2 and its virial
    // W^{F,*} = kc (1/2) sum_l w_l |rho_l|^2 (1 - k_l^2/(2 alpha))
    double s = 0.0, v = 0.0;
    for (int l = threadIdx.x; l < a.P; l += kEnergyThreads) {
      const double u = 0.5 * a.w[l] * (a.rho[l] * a.rho[l] + a.rho[a.P + l] * a.rho[a.P + l]);
      const double kx = kTwoPi * a.mkd[l] / a.L[0], ky = kTwoPi * a.mkd[a.P + l] / a.L[1],
                   kz = kTwoPi * a.mkd[2 * a.P + l] / a.L[2];
      const double k2 = kx * kx + ky * ky + kz * kz;
      s += u;
      v += u * (1.0 - k2 / (2.0 * a.alpha));
    }
    uf = block_sum(s, lds);
    wf = block_sum(v, lds);
  }
  const double q2 = sum_partials(a.sq_part, a.nb_sq, 2, 0, lds);
  const double v2 = sum_partials(a.sq_part, a.nb_sq, 2, 1, lds);
  if (threadIdx.x == 0) {
    a.out[0] = near[0];
    a.out[1] = near[1];
    a.out[2] = a.rho ? a.kc * uf : 0.0;
    a.out[3] = a.rho ? a.self_coef * q2 : 0.0;
    a.out[4] = a.half_mass * v2;
    a.out[5] = near[2];
    a.out[6] = near[3];
    a.out[7] = a.rho ? a.kc * wf : 0.0;
  }
}

int energy_part_len(int64_t n_max) {
  const int64_t nb = (n_max + kEnergyThreads - 1) / kEnergyThreads;
  return (int)(4 * nb + 2 * kEnergySqBlocks);
}

void launch_energy(const PairParams &pp, double lj4, int64_t n, const Sorted &s,
                   const int32_t *cell_start, bool near, const double *q, const double *vx, const double *vy,
                   const double *vz, double *part, EnergyFinal fin, hipStream_t st) {
  int64_t nb_near = 0;
  if (near && n > 0) {
    nb_near = (n + kEnergyThreads - 1) / kEnergyThreads;
    k_energy_near<<<(unsigned)nb_near, kEnergyThreads, 0, st>>>(pp, lj4, 2.0 * std::sqrt(pp.alpha / kPi), n, s.xq,
                                                                 cell_start, part);
  }
  double *sq_part = part + 4 * nb_near;
  int64_t nb_sq = (n + kEnergyThreads - 1) / kEnergyThreads;
  if (nb_sq > kEnergySqBlocks) nb_sq = kEnergySqBlocks;
  if (nb_sq < 1) nb_sq = 1;
  k_energy_sq<<<(unsigned)nb_sq, kEnergyThreads, 0, st>>>(n, q, vx, vy, vz, sq_part);
  fin.near_part = near ? part : nullptr;
  fin.nb_near = nb_near;
  fin.sq_part = sq_part;
  fin.nb_sq = nb_sq;
  k_energy_final<<<1, kEnergyThreads, 0, st>>>(fin);
}

}  // namespace rbe
