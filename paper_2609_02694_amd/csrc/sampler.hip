// Importance sampling of Fourier modes for the RBE estimator (Sec. 2.1,
// Eq. 9): P i.i.d. modes k = 2 pi m / L, m != 0, with probability
// proportional to exp(-k^2/(4 alpha)) (or, on request, to
// exp(-k^2/(4 alpha))/k^2, drawn by rejection from the former).
//
// The Gaussian factorizes over the axes, so each component is drawn from its
// own one-dimensional discrete Gaussian exp(-(pi m / L_d)^2 / alpha) by
// inverse CDF, and the all-zero vector is rejected. The normalizer is
// S = H_x H_y H_z - 1 with H_d the one-dimensional sums. The table keeps
// |m| <= M_d = ceil(L_d sqrt(40 alpha) / pi) (the dropped factors are below
// e^-40). Weight of a drawn mode: w = (S/P) 4 pi / (V k^2).
//
// The host and device samplers consume the same counter-based draws and the
// same table bits, so they agree bit for bit.
#include <cmath>
#include <vector>

#include "sampler_device.h"

namespace rbe {

int axis_cutoff(double L, double alpha) { return (int)std::ceil(L * std::sqrt(40.0 * alpha) / kPi); }

void build_mode_table(const double L[3], double alpha, ModeTable *t, double *cdf, int kdist) {
  int off = 0;
  double H[3];
  for (int d = 0; d < 3; ++d) {
    const int M = axis_cutoff(L[d], alpha);
    t->M[d] = M;
    t->off[d] = off;
    const int len = 2 * M + 1;
    double acc = 0.0;
    for (int i = 0; i < len; ++i) {
      const double a = kPi * (double)(i - M) / L[d];
      acc += std::exp(-(a * a) / alpha);
      if (cdf) cdf[off + i] = acc;
    }
    H[d] = acc;
    if (cdf)
      for (int i = 0; i < len; ++i) cdf[off + i] = cdf[off + i] / acc;
    off += len;
    t->L[d] = L[d];
  }
  t->total = off;
  t->S = H[0] * H[1] * H[2] - 1.0;
  t->V = L[0] * L[1] * L[2];
  t->kdist = kdist;
  t->kmin2 = 0.0;
  t->S2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double k = kTwoPi * 1.0 / L[d];
    if (d == 0 || k * k < t->kmin2) t->kmin2 = k * k;
  }
  if (kdist == RBE_KDIST_GAUSS_OVER_K2 && cdf) {
    // S2 = sum over the table's lattice without m = 0 of
    // exp(-k^2/(4 alpha))/k^2; the terms of m and -m (per axis) are equal,
    // so the octant m >= 0 is summed with multiplicity 2^(nonzero
    // components), Kahan-compensated
    std::vector<double> g[3];
    for (int d = 0; d < 3; ++d) {
      g[d].resize(t->M[d] + 1);
      for (int i = 0; i <= t->M[d]; ++i) {
        const double a = kPi * (double)i / L[d];
        g[d][i] = std::exp(-(a * a) / alpha);
      }
    }
    double sum = 0.0, comp = 0.0;
    for (int a = 0; a <= t->M[0]; ++a)
      for (int b = 0; b <= t->M[1]; ++b)
        for (int c = 0; c <= t->M[2]; ++c) {
          if (a == 0 && b == 0 && c == 0) continue;
          const double mult = (double)((a ? 2 : 1) * (b ? 2 : 1) * (c ? 2 : 1));
          const double v = mult * (g[0][a] * g[1][b] * g[2][c]) / mode_k2(*t, a, b, c);
          const double y = v - comp;
          const double s = sum + y;
          comp = (s - sum) - y;
          sum = s;
        }
    t->S2 = sum;
  }
}

int sample_modes_host(const ModeTable &t, const double *cdf, uint64_t seed, uint64_t eval, int P, int32_t *m,
                      double *w) {
  const uint64_t ek = stream_out(seed ^ kTagModes, eval);
  for (int l = 0; l < P; ++l) {
    int mv[3];
    if (!draw_mode(t, cdf, ek, l, mv)) return -1;
    m[l] = mv[0];
    m[P + l] = mv[1];
    m[2 * P + l] = mv[2];
    w[l] = mode_weight(t, P, mv[0], mv[1], mv[2]);
  }
  return 0;
}

// Evaluation eval + blockIdx.y writes its sample at m + 3P y, w + P y (and
// the mode vectors as doubles at mkd + 3P y when mkd is given).
__global__ void __launch_bounds__(256) k_sample_modes(ModeTable t, const double *__restrict__ cdf, uint64_t seed,
                                                      uint64_t eval, int P, int32_t *__restrict__ m,
                                                      double *__restrict__ w, double *__restrict__ mkd, int *err) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l >= P) return;
  const int y = blockIdx.y;
  const uint64_t ek = stream_out(seed ^ kTagModes, eval + (uint64_t)y);
  int mv[3];
  if (!draw_mode(t, cdf, ek, l, mv)) {
    atomicOr(err, kErrSampler);
    mv[0] = 1; mv[1] = 0; mv[2] = 0;
  }
  int32_t *my = m + (int64_t)3 * P * y;
  my[l] = mv[0];
  my[P + l] = mv[1];
  my[2 * P + l] = mv[2];
  w[(int64_t)P * y + l] = mode_weight(t, P, mv[0], mv[1], mv[2]);
  if (mkd) {
    double *dy = mkd + (int64_t)3 * P * y;
    dy[l] = (double)mv[0];
    dy[P + l] = (double)mv[1];
    dy[2 * P + l] = (double)mv[2];
  }
}

void launch_sample_modes(const ModeTable &t, const double *cdf_dev, uint64_t seed, uint64_t eval, int P, int32_t *m,
                         double *w, int *err_flag, hipStream_t st, int nev, double *mkd) {
  if (nev < 1) return;
  k_sample_modes<<<dim3((unsigned)((P + 255) / 256), (unsigned)nev), 256, 0, st>>>(t, cdf_dev, seed, eval, P, m, w,
                                                                                   mkd, err_flag);
}

}  // namespace rbe
