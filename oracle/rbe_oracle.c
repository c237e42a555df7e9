/*
 * rbe_oracle.c -- TEST INFRASTRUCTURE ONLY: plain FP64 CPU reference for the
 * random batch Ewald nonbonded force of RBMD 2.0 (arXiv 2609.02694).
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library. It shares no code with the GPU
 * library; the two meet only through the seeded inputs and the documented
 * counter-based generator definitions restated below.
 *
 * Every routine is the plain definition written out: no blocking, no fusion,
 * loops in the order of the paper's sums. Parallel loops (OpenMP) split the
 * OUTER index only, so each reduced value has one fixed summation order.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off (no FMA contraction: the wrapped
 * coordinates, squared distances and cutoff classifications must be the
 * exact IEEE results of the written expressions).
 *
 * Sign conventions (readings of the paper):
 *  - Near field (Sec. 2.1, Eq. 7-8): F_i = -grad_i U gives
 *    F_i^N = + sum_j (q_i q_j G(r) + G_LJ(r)) (r_i - r_j) for the minimum image;
 *    the printed leading minus of Eq. 7 is taken as a typo (checked here by
 *    finite differences of the real-space energy in the tests).
 *  - RBE estimator (Eq. 9): keeps the minus sign of the exact Fourier force of
 *    Eq. 7, F_i = -(S/P) sum_l 4 pi q_i k_l/(V k_l^2) Im(exp(-i k_l.r_i) rho_l).
 */
#include "rbe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define PI 3.14159265358979323846264338327950288
#define TWO_PI 6.28318530717958647692528676655900577

int orc_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Threads of the parallel loops that follow (timing only: every loop here
   partitions its work deterministically, so the results do not change). */
void orc_set_num_threads(int k) {
#ifdef _OPENMP
  if (k > 0) omp_set_num_threads(k);
#else
  (void)k;
#endif
}

/* ===================================================================== */
/* Counter-based generators                                               */
/* ===================================================================== */
/* SplitMix64 (Steele, Lea & Flood 2014): output n of the stream seeded by s
   is mix64(s + (n+1) * GAMMA). */
#define GAMMA 0x9E3779B97F4A7C15ULL
#define TAG_KSET 0x4B4D4F4445534554ULL /* "KMODESET" */
#define TAG_RBL 0x52424C5348454C4CULL  /* "RBLSHELL" */

uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static uint64_t sm_out(uint64_t s, uint64_t n) { return orc_mix64(s + (n + 1) * GAMMA); }
static double u53(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

/* lowbias32 (C. Wellons, hash-prospector): a bijection of 32-bit integers.
   Parity unpinned: no published output of it is at hand; the tests pin its
   bijectivity and the unbiasedness of the batches it selects, and the GPU
   must reproduce it bit for bit. */
static uint32_t lowbias32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x7feb352dU;
  x ^= x >> 15;
  x *= 0x846ca68bU;
  x ^= x >> 16;
  return x;
}

/* Shell ranking key for the pair (i, j) at force evaluation `eval`:
   h = output id_i of the stream seeded by output `eval` of the stream seeded
   by seed ^ TAG_RBL; key = lowbias32(lowbias32(id_j ^ lo32(h)) ^ hi32(h)).
   For fixed (seed, eval, i) the key is a bijection of id_j, so distinct
   particles never tie. */
uint32_t orc_rbl_key(uint64_t seed, uint64_t eval, int32_t id_i, int32_t id_j) {
  uint64_t k = sm_out(seed ^ TAG_RBL, eval);
  uint64_t h = sm_out(k, (uint64_t)(uint32_t)id_i);
  uint32_t a = (uint32_t)h, b = (uint32_t)(h >> 32);
  return lowbias32(lowbias32((uint32_t)id_j ^ a) ^ b);
}

/* ===================================================================== */
/* Fourier-mode sampling: P(k) ~ exp(-k^2/(4 alpha)) on K \ {0} (Eq. 9)   */
/* ===================================================================== */
/* The lattice is k = 2 pi m / L (Eq. 5). Per axis, exp(-k_d^2/(4 alpha)) =
   exp(-(pi m / L_d)^2 / alpha). The table keeps |m| <= M with
   M = ceil(L sqrt(40 alpha) / pi): beyond it the factor is below exp(-40). */
int orc_axis_cutoff(double L, double alpha) { return (int)ceil(L * sqrt(40.0 * alpha) / PI); }

static double axis_weight(int m, double L, double alpha) {
  double t = PI * (double)m / L;
  return exp(-(t * t) / alpha);
}

/* H_d = sum_m exp(-(pi m/L)^2/alpha), summed from m = -M upwards. */
double orc_axis_H(double L, double alpha) {
  int M = orc_axis_cutoff(L, alpha);
  double h = 0.0;
  for (int m = -M; m <= M; ++m) h += axis_weight(m, L, alpha);
  return h;
}

/* Normalizer of Eq. 9: S = sum_{k != 0} exp(-k^2/4a) = H_x H_y H_z - 1
   (the Gaussian factorizes over the axes; the k = 0 term is 1). */
double orc_norm_S(const double L[3], double alpha) {
  return orc_axis_H(L[0], alpha) * orc_axis_H(L[1], alpha) * orc_axis_H(L[2], alpha) - 1.0;
}

/* k^2 of the mode m (k = 2 pi m / L), summed x, y, z. */
static double mode_k2(const int mv[3], const double L[3]) {
  double k2 = 0.0;
  for (int d = 0; d < 3; ++d) {
    double kd = TWO_PI * (double)mv[d] / L[d];
    k2 += kd * kd;
  }
  return k2;
}

/* Normalizer of the alternative proposal P(k) ~ exp(-k^2/4a)/k^2:
   S2 = sum over the sampler's lattice (|m_d| <= M_d, m != 0) of
   exp(-k^2/4a)/k^2, the Gaussian factor as the product of the axis factors.
   The sum runs over up to 10^8 positive terms, so it is compensated (Kahan,
   same order): plain summation would leave an error of order 1e-11 in
   every weight. */
double orc_norm_S2(const double L[3], double alpha) {
  int M[3];
  for (int d = 0; d < 3; ++d) M[d] = orc_axis_cutoff(L[d], alpha);
  double s = 0.0, comp = 0.0;
  for (int a = -M[0]; a <= M[0]; ++a)
    for (int b = -M[1]; b <= M[1]; ++b)
      for (int c = -M[2]; c <= M[2]; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        const int mv[3] = {a, b, c};
        double g = axis_weight(a, L[0], alpha) * axis_weight(b, L[1], alpha) * axis_weight(c, L[2], alpha);
        double y = g / mode_k2(mv, L) - comp;
        double t = s + y;
        comp = (t - s) - y;
        s = t;
      }
  return s;
}

/* Draw of mode l at evaluation `eval`: attempt a uses draws 3a, 3a+1, 3a+2 of
   the stream seeded by K_{e,l} = output l of the stream seeded by
   K_e = output eval of the stream seeded by seed ^ TAG_KSET. Each draw u is
   mapped to m = the first table entry whose cumulative probability exceeds u
   (inverse CDF). The all-zero vector is rejected (next attempt).
   kdist = 1, P(k) ~ exp(-k^2/4a)/k^2: attempt a uses draws 4a..4a+2 that way
   and draw 4a+3 = u; it is accepted when m != 0 and u k^2 < k_min^2,
   k_min^2 = min_d (2 pi / L_d)^2 (so a Gaussian proposal m is kept with
   probability k_min^2/k^2, which leaves exp(-k^2/4a)/k^2). Weights:
   (S2/P) 4 pi / V. */
int orc_sample_k(uint64_t seed, uint64_t eval, const double L[3], double alpha, int32_t P, int32_t kdist,
                 int32_t *m, double *w) {
  if (P <= 0 || !(alpha > 0) || (kdist != 0 && kdist != 1)) return -1;
  int M[3];
  double *cdf[3];
  double H[3];
  for (int d = 0; d < 3; ++d) {
    M[d] = orc_axis_cutoff(L[d], alpha);
    int len = 2 * M[d] + 1;
    cdf[d] = (double *)malloc(sizeof(double) * len);
    double acc = 0.0;
    for (int i = 0; i < len; ++i) {
      acc += axis_weight(i - M[d], L[d], alpha);
      cdf[d][i] = acc;
    }
    H[d] = acc;
    for (int i = 0; i < len; ++i) cdf[d][i] = cdf[d][i] / H[d];
  }
  const double S = H[0] * H[1] * H[2] - 1.0;
  const double V = L[0] * L[1] * L[2];
  double kmin2 = 0.0, S2 = 0.0;
  if (kdist == 1) {
    for (int d = 0; d < 3; ++d) {
      double k = TWO_PI * 1.0 / L[d];
      if (d == 0 || k * k < kmin2) kmin2 = k * k;
    }
    S2 = orc_norm_S2(L, alpha);
  }
  const int per = kdist == 1 ? 4 : 3;
  const long cap = kdist == 1 ? (1L << 20) : 4096;
  uint64_t ke = sm_out(seed ^ TAG_KSET, eval);
  int status = 0;
  for (int32_t l = 0; l < P; ++l) {
    uint64_t kl = sm_out(ke, (uint64_t)l);
    int mv[3] = {0, 0, 0};
    int ok = 0;
    for (long a = 0; a < cap && !ok; ++a) {
      for (int d = 0; d < 3; ++d) {
        double u = u53(sm_out(kl, (uint64_t)(per * a + d)));
        int len = 2 * M[d] + 1;
        int i = 0;
        while (i < len - 1 && !(u < cdf[d][i])) ++i; /* first entry with u < cdf */
        mv[d] = i - M[d];
      }
      ok = (mv[0] != 0 || mv[1] != 0 || mv[2] != 0);
      if (ok && kdist == 1) {
        double u = u53(sm_out(kl, (uint64_t)(per * a + 3)));
        ok = u * mode_k2(mv, L) < kmin2;
      }
    }
    if (!ok) { status = -2; break; }
    m[l] = mv[0];
    m[P + l] = mv[1];
    m[2 * P + l] = mv[2];
    if (kdist == 1) w[l] = (S2 / (double)P) * (4.0 * PI / V);
    else w[l] = (S / (double)P) * (4.0 * PI / (V * mode_k2(mv, L)));
  }
  for (int d = 0; d < 3; ++d) free(cdf[d]);
  return status;
}

/* ===================================================================== */
/* Periodic wrap                                                          */
/* ===================================================================== */
static double wrap1(double x, double L) {
  double w = x - L * floor(x / L);
  if (w < 0.0 || w >= L) w = 0.0; /* only reached through rounding */
  return w;
}

/* ===================================================================== */
/* Structure factor and Fourier force for a given mode set                */
/* ===================================================================== */
/* Phase of particle j for mode l: theta = k_l . r_j = 2 pi (m . s_j) with the
   fractional coordinate s = r/L. Whole turns are removed before the sine and
   cosine: theta = 2 pi (t - rint(t)), t = m.s (the same angle modulo 2 pi). */
static double phase(const int32_t *m, int32_t P, int32_t l, double sx, double sy, double sz) {
  double t = (double)m[l] * sx + (double)m[P + l] * sy + (double)m[2 * P + l] * sz;
  t = t - rint(t);
  return TWO_PI * t;
}

/* rho(k_l) = sum_j q_j exp(i k_l . r_j)  (Eq. 5) */
void orc_rho(int64_t n, const double *x, const double *y, const double *z, const double *q, const double L[3],
             int32_t P, const int32_t *m, double *rho_re, double *rho_im) {
#pragma omp parallel for schedule(static)
  for (int32_t l = 0; l < P; ++l) {
    double re = 0.0, im = 0.0;
    for (int64_t j = 0; j < n; ++j) {
      if (q[j] == 0.0) continue;
      double th = phase(m, P, l, wrap1(x[j], L[0]) / L[0], wrap1(y[j], L[1]) / L[1], wrap1(z[j], L[2]) / L[2]);
      re += q[j] * cos(th);
      im += q[j] * sin(th);
    }
    rho_re[l] = re;
    rho_im[l] = im;
  }
}

/* F_i = -q_i sum_l w_l k_l Im(exp(-i k_l.r_i) rho_l),
   Im(exp(-i th) rho) = cos(th) Im(rho) - sin(th) Re(rho)   (Eq. 7 and 9) */
void orc_fourier_force(int64_t n, const double *x, const double *y, const double *z, const double *q,
                       const double L[3], int32_t P, const int32_t *m, const double *w, const double *rho_re,
                       const double *rho_im, double *fx, double *fy, double *fz) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    double gx = 0.0, gy = 0.0, gz = 0.0;
    if (q[i] != 0.0) {
      double sx = wrap1(x[i], L[0]) / L[0], sy = wrap1(y[i], L[1]) / L[1], sz = wrap1(z[i], L[2]) / L[2];
      for (int32_t l = 0; l < P; ++l) {
        double th = phase(m, P, l, sx, sy, sz);
        double im_part = cos(th) * rho_im[l] - sin(th) * rho_re[l];
        double g = w[l] * im_part;
        gx += g * (TWO_PI * (double)m[l] / L[0]);
        gy += g * (TWO_PI * (double)m[P + l] / L[1]);
        gz += g * (TWO_PI * (double)m[2 * P + l] / L[2]);
      }
      gx *= -q[i];
      gy *= -q[i];
      gz *= -q[i];
    }
    fx[i] = gx;
    fy[i] = gy;
    fz[i] = gz;
  }
}

double orc_fourier_energy(int32_t P, const double *w, const double *rho_re, const double *rho_im) {
  double u = 0.0;
  for (int32_t l = 0; l < P; ++l) u += 0.5 * w[l] * (rho_re[l] * rho_re[l] + rho_im[l] * rho_im[l]);
  return u;
}

/* Virial of the fixed-mode energy U* under a uniform dilation of positions
   and box (k_l -> k_l/s, V -> s^3 V, rho_l unchanged), with the sampling
   weights read as the importance-sampled sum of Eq. 5:
   W = -dU/ds = (1/2) sum_l w_l |rho_l|^2 (1 - k_l^2/(2 alpha)). */
double orc_fourier_virial(int32_t P, const int32_t *m, const double L[3], double alpha, const double *w,
                          const double *rho_re, const double *rho_im) {
  double v = 0.0;
  for (int32_t l = 0; l < P; ++l) {
    double kx = TWO_PI * m[l] / L[0], ky = TWO_PI * m[P + l] / L[1], kz = TWO_PI * m[2 * P + l] / L[2];
    double k2 = kx * kx + ky * ky + kz * kz;
    v += 0.5 * w[l] * (rho_re[l] * rho_re[l] + rho_im[l] * rho_im[l]) * (1.0 - k2 / (2.0 * alpha));
  }
  return v;
}

/* ===================================================================== */
/* Real space: erfc-Coulomb + LJ with the random batch list              */
/* ===================================================================== */
/* G(r) = erfc(sqrt(a) r)/r^3 + 2 sqrt(a) exp(-a r^2)/(sqrt(pi) r^2)   (Eq. 8)
   G_LJ(r) = 24 eps (2 sigma^12/r^14 - sigma^6/r^8)                   (Eq. 8)
   pair force on i: (kc q_i q_j G + G_LJ) * d, d = r_i - r_j (min image). */
typedef struct {
  double rc2, rlj2, rcore2, sa, kc, eps, sig2;
  int terms;
  int shell_charged;
} pair_consts;

static pair_consts make_consts(const orc_sys *s, int32_t terms) {
  pair_consts c;
  c.rc2 = s->r_coul * s->r_coul;
  c.rlj2 = s->r_lj * s->r_lj;
  c.rcore2 = s->r_core * s->r_core;
  c.sa = sqrt(s->alpha);
  c.kc = s->kc;
  c.eps = s->eps;
  c.sig2 = s->sigma * s->sigma;
  c.terms = terms;
  c.shell_charged = s->shell_charged;
  return c;
}

/* scalar factor f such that the pair force on i is f * d */
static double pair_scalar(const pair_consts *c, double r2, double qi, double qj) {
  double f = 0.0;
  if ((c->terms & ORC_COUL_REAL) && r2 <= c->rc2 && qi != 0.0 && qj != 0.0) {
    double r = sqrt(r2);
    double G = erfc(c->sa * r) / (r2 * r) + 2.0 * c->sa * exp(-(c->sa * c->sa) * r2) / (sqrt(PI) * r2);
    f += c->kc * qi * qj * G;
  }
  if ((c->terms & ORC_LJ) && r2 <= c->rlj2) {
    double s2 = c->sig2 / r2;
    double s6 = s2 * s2 * s2;
    f += 24.0 * c->eps * (2.0 * s6 * s6 - s6) / r2;
  }
  return f;
}

static void min_image(const double L[3], double xi, double yi, double zi, double xj, double yj, double zj,
                      double *dx, double *dy, double *dz) {
  double ax = xi - xj, ay = yi - yj, az = zi - zj;
  *dx = ax - L[0] * rint(ax / L[0]);
  *dy = ay - L[1] * rint(ay / L[1]);
  *dz = az - L[2] * rint(az / L[2]);
}

typedef struct {
  uint32_t key;
  int64_t j;
  double dx, dy, dz, r2;
} shell_entry;

static int cmp_shell(const void *a, const void *b) {
  uint32_t ka = ((const shell_entry *)a)->key, kb = ((const shell_entry *)b)->key;
  return ka < kb ? -1 : (ka > kb ? 1 : 0);
}

/* Does particle i need the shell of Eq. 11? Its shell terms are identically
   zero when q_i = 0 and the LJ cutoff lies inside the core. */
static int rbl_active(const orc_sys *s, double qi) {
  return s->r_core > 0.0 && s->p_shell > 0 && (qi != 0.0 || s->r_lj > s->r_core);
}

/* Growable per-thread shell buffer */
typedef struct {
  shell_entry *e;
  int64_t n, cap;
} shell_buf;
static void shell_push(shell_buf *b, shell_entry v) {
  if (b->n == b->cap) {
    b->cap = b->cap ? 2 * b->cap : 1024;
    b->e = (shell_entry *)realloc(b->e, sizeof(shell_entry) * b->cap);
  }
  b->e[b->n++] = v;
}

/* Visit one candidate j for particle i. */
static void visit(const pair_consts *c, int active, double qi, double qj, uint32_t key_j, int64_t j, double dx,
                  double dy, double dz, double *f, shell_buf *sb) {
  double r2 = dx * dx + dy * dy + dz * dz;
  if (active) {
    if (r2 <= c->rcore2) { /* core set C_i: exact (Eq. 10-11) */
      double g = pair_scalar(c, r2, qi, qj);
      f[0] += g * dx; f[1] += g * dy; f[2] += g * dz;
    } else if (r2 <= c->rc2 && (!c->shell_charged || qj != 0.0)) { /* shell set S_i */
      shell_entry e = {key_j, j, dx, dy, dz, r2};
      shell_push(sb, e);
    } /* else: a neutral j beyond the core of a charged-only shell, whose
         force is zero (no charge, and r > r_core >= r_lj) */
  } else {
    double g = pair_scalar(c, r2, qi, qj);
    f[0] += g * dx; f[1] += g * dy; f[2] += g * dz;
  }
}

/* Shell estimator of Eq. 11: the batch B_i is the p members of S_i with the
   smallest ranking key (all of S_i if #S_i <= p); terms scaled by #S_i/|B_i|. */
static void finish_shell(const pair_consts *c, int p, double qi, const double *q, shell_buf *sb, double *f) {
  if (sb->n == 0) return;
  qsort(sb->e, (size_t)sb->n, sizeof(shell_entry), cmp_shell);
  int64_t nb = sb->n < p ? sb->n : p;
  double scale = (double)sb->n / (double)nb;
  double g[3] = {0.0, 0.0, 0.0};
  for (int64_t b = 0; b < nb; ++b) {
    shell_entry *e = &sb->e[b];
    double s = pair_scalar(c, e->r2, qi, q[e->j]);
    g[0] += s * e->dx; g[1] += s * e->dy; g[2] += s * e->dz;
  }
  f[0] += scale * g[0]; f[1] += scale * g[1]; f[2] += scale * g[2];
}

void orc_real_force(int64_t n, const double *x, const double *y, const double *z, const double *q,
                    const int32_t *id, const orc_sys *s, int32_t terms, uint64_t seed, uint64_t eval,
                    int64_t nidx, const int64_t *idx, double *fx, double *fy, double *fz, int64_t *n_shell) {
  pair_consts c = make_consts(s, terms);
  int64_t count = idx ? nidx : n;
#pragma omp parallel
  {
    shell_buf sb = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 16)
    for (int64_t t = 0; t < count; ++t) {
      int64_t i = idx ? idx[t] : t;
      int active = rbl_active(s, q[i]);
      double f[3] = {0.0, 0.0, 0.0};
      sb.n = 0;
      for (int64_t j = 0; j < n; ++j) {
        if (j == i) continue;
        double dx, dy, dz;
        min_image(s->L, x[i], y[i], z[i], x[j], y[j], z[j], &dx, &dy, &dz);
        uint32_t key = active ? orc_rbl_key(seed, eval, id[i], id[j]) : 0u;
        visit(&c, active, q[i], q[j], key, j, dx, dy, dz, f, &sb);
      }
      if (n_shell) n_shell[t] = active ? sb.n : -1;
      if (active) finish_shell(&c, s->p_shell, q[i], q, &sb, f);
      fx[t] = f[0];
      fy[t] = f[1];
      fz[t] = f[2];
    }
    free(sb.e);
  }
}

/* Outputs of orc_real_force / orc_real_force_cells are indexed by position in
   idx (by particle when idx == NULL). */

/* Same sums through a cell grid: cells of edge >= the largest cutoff, 27
   neighbours, minimum image as above. Falls back to brute force when the
   grid has fewer than 3 cells along an axis. */
int orc_real_force_cells(int64_t n, const double *x, const double *y, const double *z, const double *q,
                         const int32_t *id, const orc_sys *s, int32_t terms, uint64_t seed, uint64_t eval,
                         int64_t nidx, const int64_t *idx, double *fx, double *fy, double *fz) {
  double rmax = s->r_coul > s->r_lj ? s->r_coul : s->r_lj;
  int nc[3];
  for (int d = 0; d < 3; ++d) {
    nc[d] = (int)floor(s->L[d] / rmax);
    if (nc[d] > 1024) nc[d] = 1024;
  }
  if (nc[0] < 3 || nc[1] < 3 || nc[2] < 3) {
    orc_real_force(n, x, y, z, q, id, s, terms, seed, eval, nidx, idx, fx, fy, fz, NULL);
    return 1;
  }
  int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ncell);
  int64_t *next = (int64_t *)malloc(sizeof(int64_t) * n);
  int *cell = (int *)malloc(sizeof(int) * 3 * n);
  if (!head || !next || !cell) { free(head); free(next); free(cell); return -1; }
  for (int64_t k = 0; k < ncell; ++k) head[k] = -1;
  for (int64_t j = n - 1; j >= 0; --j) {
    const double r[3] = {x[j], y[j], z[j]};
    for (int d = 0; d < 3; ++d) {
      int cd = (int)(wrap1(r[d], s->L[d]) / s->L[d] * nc[d]);
      cell[3 * j + d] = cd >= nc[d] ? nc[d] - 1 : cd;
    }
    int64_t k = ((int64_t)cell[3 * j + 2] * nc[1] + cell[3 * j + 1]) * nc[0] + cell[3 * j];
    next[j] = head[k];
    head[k] = j;
  }
  pair_consts c = make_consts(s, terms);
  int64_t count = idx ? nidx : n;
#pragma omp parallel
  {
    shell_buf sb = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 64)
    for (int64_t t = 0; t < count; ++t) {
      int64_t i = idx ? idx[t] : t;
      int active = rbl_active(s, q[i]);
      double f[3] = {0.0, 0.0, 0.0};
      sb.n = 0;
      for (int oz = -1; oz <= 1; ++oz)
        for (int oy = -1; oy <= 1; ++oy)
          for (int ox = -1; ox <= 1; ++ox) {
            int cx = (cell[3 * i] + ox + nc[0]) % nc[0];
            int cy = (cell[3 * i + 1] + oy + nc[1]) % nc[1];
            int cz = (cell[3 * i + 2] + oz + nc[2]) % nc[2];
            for (int64_t j = head[((int64_t)cz * nc[1] + cy) * nc[0] + cx]; j >= 0; j = next[j]) {
              if (j == i) continue;
              double dx, dy, dz;
              min_image(s->L, x[i], y[i], z[i], x[j], y[j], z[j], &dx, &dy, &dz);
              uint32_t key = active ? orc_rbl_key(seed, eval, id[i], id[j]) : 0u;
              visit(&c, active, q[i], q[j], key, j, dx, dy, dz, f, &sb);
            }
          }
      if (active) finish_shell(&c, s->p_shell, q[i], q, &sb, f);
      fx[t] = f[0];
      fy[t] = f[1];
      fz[t] = f[2];
    }
    free(sb.e);
  }
  free(head);
  free(next);
  free(cell);
  return 0;
}

/* Eq. 12: F_i <- F_i - (1/N) sum_j F_j */
void orc_mean_correct(int64_t n, double *fx, double *fy, double *fz, double mean_out[3]) {
  double s[3] = {0.0, 0.0, 0.0};
  for (int64_t i = 0; i < n; ++i) { s[0] += fx[i]; s[1] += fy[i]; s[2] += fz[i]; }
  for (int d = 0; d < 3; ++d) s[d] /= (double)n;
  for (int64_t i = 0; i < n; ++i) { fx[i] -= s[0]; fy[i] -= s[1]; fz[i] -= s[2]; }
  if (mean_out) { mean_out[0] = s[0]; mean_out[1] = s[1]; mean_out[2] = s[2]; }
}

/* U_N = sum_{i<j} kc q_i q_j erfc(sqrt(a) r)/r (r <= r_coul),
   U_LJ = sum_{i<j} 4 eps ((sigma/r)^12 - (sigma/r)^6) (r <= r_lj). */
void orc_real_energy(int64_t n, const double *x, const double *y, const double *z, const double *q,
                     const orc_sys *s, double *u_coul, double *u_lj) {
  double uc = 0.0, ul = 0.0;
  const double rc2 = s->r_coul * s->r_coul, rl2 = s->r_lj * s->r_lj, sa = sqrt(s->alpha);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : uc, ul)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i + 1; j < n; ++j) {
      double dx, dy, dz;
      min_image(s->L, x[i], y[i], z[i], x[j], y[j], z[j], &dx, &dy, &dz);
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 <= rc2) {
        double r = sqrt(r2);
        uc += s->kc * q[i] * q[j] * erfc(sa * r) / r;
      }
      if (r2 <= rl2) {
        double s2 = s->sigma * s->sigma / r2, s6 = s2 * s2 * s2;
        ul += 4.0 * s->eps * (s6 * s6 - s6);
      }
    }
  }
  *u_coul = uc;
  *u_lj = ul;
}

/* Pair virials W = sum_{i<j} d_ij . F_ij (d = r_i - r_j, minimum image):
   Coulomb: kc q_i q_j r^2 G(r) (r <= r_coul), LJ: r^2 G_LJ(r) (r <= r_lj),
   with G and G_LJ of Eq. 8. */
void orc_real_virial(int64_t n, const double *x, const double *y, const double *z, const double *q,
                     const orc_sys *s, double *w_coul, double *w_lj) {
  double wc = 0.0, wl = 0.0;
  const double rc2 = s->r_coul * s->r_coul, rl2 = s->r_lj * s->r_lj, sa = sqrt(s->alpha);
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : wc, wl)
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t j = i + 1; j < n; ++j) {
      double dx, dy, dz;
      min_image(s->L, x[i], y[i], z[i], x[j], y[j], z[j], &dx, &dy, &dz);
      double r2 = dx * dx + dy * dy + dz * dz;
      if (r2 <= rc2) {
        double r = sqrt(r2);
        double G = erfc(sa * r) / (r2 * r) + 2.0 * sa * exp(-s->alpha * r2) / (sqrt(PI) * r2);
        wc += s->kc * q[i] * q[j] * G * r2;
      }
      if (r2 <= rl2) {
        double s2 = s->sigma * s->sigma / r2, s6 = s2 * s2 * s2;
        double GL = 24.0 * s->eps * (2.0 * s6 * s6 - s6) / r2;
        wl += GL * r2;
      }
    }
  }
  *w_coul = wc;
  *w_lj = wl;
}

/* ===================================================================== */
/* Exact Ewald sum (tiny boxes)                                           */
/* ===================================================================== */
/* Real part: U = 1/2 sum'_{n,i,j} q_i q_j erfc(sqrt(a)|r_ij + nL|)/|r_ij + nL|
   over every image with erfc(sqrt(a) r) >= tol. Reciprocal part (Eq. 5):
   U^F = (2 pi/V) sum_{k != 0} |rho(k)|^2 exp(-k^2/4a)/k^2 over every mode
   whose per-axis Gaussian factors stay above tol (bound on |m_d| below).
   Self energy (Eq. 6): sqrt(a/pi) sum q_i^2. Forces: Eq. 7 with the sign
   reading above. Outputs are indexed like the inputs. */
void orc_ewald_exact(int64_t n, const double *x, const double *y, const double *z, const double *q,
                     const double L[3], double alpha, double tol, double *u_real, double *u_recip, double *u_self,
                     double *fx, double *fy, double *fz) {
  const double sa = sqrt(alpha);
  double xr = 0.0; /* erfc(xr) < tol */
  while (erfc(xr) >= tol) xr += 0.01;
  const double rmax = xr / sa;
  int nmax[3];
  for (int d = 0; d < 3; ++d) nmax[d] = (int)ceil(rmax / L[d]) + 1;
  double ur = 0.0;
  for (int64_t i = 0; i < n; ++i) { fx[i] = 0.0; fy[i] = 0.0; fz[i] = 0.0; }
#pragma omp parallel for schedule(dynamic, 1) reduction(+ : ur)
  for (int64_t i = 0; i < n; ++i) {
    double f[3] = {0.0, 0.0, 0.0};
    for (int64_t j = 0; j < n; ++j)
      for (int a = -nmax[0]; a <= nmax[0]; ++a)
        for (int b = -nmax[1]; b <= nmax[1]; ++b)
          for (int c = -nmax[2]; c <= nmax[2]; ++c) {
            if (j == i && a == 0 && b == 0 && c == 0) continue;
            double dx = x[i] - x[j] + a * L[0], dy = y[i] - y[j] + b * L[1], dz = z[i] - z[j] + c * L[2];
            double r2 = dx * dx + dy * dy + dz * dz, r = sqrt(r2);
            if (r > rmax) continue;
            ur += 0.5 * q[i] * q[j] * erfc(sa * r) / r;
            double G = erfc(sa * r) / (r2 * r) + 2.0 * sa * exp(-alpha * r2) / (sqrt(PI) * r2);
            f[0] += q[i] * q[j] * G * dx;
            f[1] += q[i] * q[j] * G * dy;
            f[2] += q[i] * q[j] * G * dz;
          }
    fx[i] += f[0];
    fy[i] += f[1];
    fz[i] += f[2];
  }
  /* reciprocal: exp(-pi^2 m^2/(a L^2)) >= tol  ->  |m| <= L sqrt(a ln(1/tol))/pi */
  int mm[3];
  for (int d = 0; d < 3; ++d) mm[d] = (int)ceil(L[d] * sqrt(alpha * log(1.0 / tol)) / PI) + 1;
  const double V = L[0] * L[1] * L[2];
  double uk = 0.0;
  double *gx = (double *)calloc((size_t)n, sizeof(double));
  double *gy = (double *)calloc((size_t)n, sizeof(double));
  double *gz = (double *)calloc((size_t)n, sizeof(double));
  for (int a = -mm[0]; a <= mm[0]; ++a)
    for (int b = -mm[1]; b <= mm[1]; ++b)
      for (int c = -mm[2]; c <= mm[2]; ++c) {
        if (a == 0 && b == 0 && c == 0) continue;
        double kx = TWO_PI * a / L[0], ky = TWO_PI * b / L[1], kz = TWO_PI * c / L[2];
        double k2 = kx * kx + ky * ky + kz * kz;
        double damp = exp(-k2 / (4.0 * alpha));
        if (damp < tol * 1e-3) continue;
        double re = 0.0, im = 0.0;
        for (int64_t j = 0; j < n; ++j) {
          double th = kx * x[j] + ky * y[j] + kz * z[j];
          re += q[j] * cos(th);
          im += q[j] * sin(th);
        }
        uk += (2.0 * PI / V) * (re * re + im * im) / k2 * damp;
        double pref = 4.0 * PI / (V * k2) * damp;
        for (int64_t i = 0; i < n; ++i) {
          double th = kx * x[i] + ky * y[i] + kz * z[i];
          /* Im(exp(-i th) rho) */
          double s = cos(th) * im - sin(th) * re;
          gx[i] -= pref * q[i] * kx * s;
          gy[i] -= pref * q[i] * ky * s;
          gz[i] -= pref * q[i] * kz * s;
        }
      }
  for (int64_t i = 0; i < n; ++i) { fx[i] += gx[i]; fy[i] += gy[i]; fz[i] += gz[i]; }
  free(gx); free(gy); free(gz);
  *u_real = ur;
  *u_recip = uk;
  *u_self = orc_self_energy(n, q, alpha);
}

/* Self energy (Eq. 6): sqrt(a/pi) sum_i q_i^2. */
double orc_self_energy(int64_t n, const double *q, double alpha) {
  double us = 0.0;
  for (int64_t i = 0; i < n; ++i) us += q[i] * q[i];
  return us * sqrt(alpha / PI);
}

/* Kinetic energy (m/2) sum_i |v_i|^2. */
double orc_kinetic_energy(int64_t n, const double *vx, const double *vy, const double *vz, double mass) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += vx[i] * vx[i] + vy[i] * vy[i] + vz[i] * vz[i];
  return 0.5 * mass * s;
}

int64_t orc_full_lattice(const double L[3], double alpha, const int32_t mmax[3], int32_t *m, double *w) {
  int64_t cnt = 0;
  for (int a = -mmax[0]; a <= mmax[0]; ++a)
    for (int b = -mmax[1]; b <= mmax[1]; ++b)
      for (int c = -mmax[2]; c <= mmax[2]; ++c)
        if (a || b || c) ++cnt;
  if (!m || !w) return cnt;
  const double V = L[0] * L[1] * L[2];
  int64_t l = 0;
  for (int a = -mmax[0]; a <= mmax[0]; ++a)
    for (int b = -mmax[1]; b <= mmax[1]; ++b)
      for (int c = -mmax[2]; c <= mmax[2]; ++c) {
        if (!(a || b || c)) continue;
        double kx = TWO_PI * a / L[0], ky = TWO_PI * b / L[1], kz = TWO_PI * c / L[2];
        double k2 = kx * kx + ky * ky + kz * kz;
        m[l] = a;
        m[cnt + l] = b;
        m[2 * cnt + l] = c;
        w[l] = 4.0 * PI * exp(-k2 / (4.0 * alpha)) / (V * k2);
        ++l;
      }
  return cnt;
}

/* ===================================================================== */
/* Cell binning                                                           */
/* ===================================================================== */
/* key = species * ncell + (c_z * n_y + c_y) * n_x + c_x, species 0 for
   charged and 1 for neutral particles, c_d = min(n_d - 1, floor(w_d * (n_d/L_d)))
   with w the wrapped coordinate. Stable counting sort: perm lists particle
   indices in key order, ties in input order; cell_start[k] is the first slot
   of key k (2*ncell + 1 entries). */
int orc_bin(int64_t n, const double *x, const double *y, const double *z, const double *q, const double L[3],
            const int32_t ncell[3], int32_t *cell_start, int32_t *perm) {
  const int64_t nc = (int64_t)ncell[0] * ncell[1] * ncell[2];
  const int64_t nkeys = 2 * nc;
  double scale[3];
  for (int d = 0; d < 3; ++d) scale[d] = (double)ncell[d] / L[d];
  int64_t *key = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  int64_t *cnt = (int64_t *)calloc((size_t)nkeys + 1, sizeof(int64_t));
  if (!key || !cnt) { free(key); free(cnt); return -1; }
  for (int64_t i = 0; i < n; ++i) {
    const double r[3] = {x[i], y[i], z[i]};
    int64_t c[3];
    for (int d = 0; d < 3; ++d) {
      int64_t cd = (int64_t)(wrap1(r[d], L[d]) * scale[d]);
      c[d] = cd >= ncell[d] ? ncell[d] - 1 : cd;
    }
    key[i] = (q[i] == 0.0 ? nc : 0) + (c[2] * ncell[1] + c[1]) * ncell[0] + c[0];
    cnt[key[i]]++;
  }
  int64_t acc = 0;
  for (int64_t k = 0; k < nkeys; ++k) {
    int64_t c = cnt[k];
    cell_start[k] = (int32_t)acc;
    cnt[k] = acc;
    acc += c;
  }
  cell_start[nkeys] = (int32_t)acc;
  for (int64_t i = 0; i < n; ++i) perm[cnt[key[i]]++] = (int32_t)i;
  free(key);
  free(cnt);
  return 0;
}

/* ===================================================================== */
/* Velocity Verlet pieces                                                 */
/* ===================================================================== */
void orc_kick(int64_t n, double half_dt_over_m, const double *fx, const double *fy, const double *fz, double *vx,
              double *vy, double *vz) {
  for (int64_t i = 0; i < n; ++i) {
    vx[i] += half_dt_over_m * fx[i];
    vy[i] += half_dt_over_m * fy[i];
    vz[i] += half_dt_over_m * fz[i];
  }
}

void orc_drift_wrap(int64_t n, double dt, const double L[3], const double *vx, const double *vy, const double *vz,
                    double *x, double *y, double *z) {
  for (int64_t i = 0; i < n; ++i) {
    x[i] = wrap1(x[i] + dt * vx[i], L[0]);
    y[i] = wrap1(y[i] + dt * vy[i], L[1]);
    z[i] = wrap1(z[i] + dt * vz[i], L[2]);
  }
}
