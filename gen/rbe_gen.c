/*
 * Seeded synthetic inputs for charged Lennard-Jones systems.
 *
 * This module holds no arithmetic of the random batch Ewald method: it only
 * draws particle positions, charges and velocities. Both the CPU oracle and
 * the GPU library consume its output as plain arrays.
 *
 * Random numbers: a counter-based SplitMix64 stream (Steele, Lea & Flood,
 * "Fast splittable pseudorandom number generators", OOPSLA 2014). Output n of
 * the stream with seed s is mix64(s + (n+1)*GAMMA).
 *
 * Positions: random sequential addition (RSA). Particle i proposes uniform
 * points in the periodic box and keeps the first one whose minimum-image
 * distance to every earlier particle is at least d_min. This avoids the
 * near-overlaps that plain uniform sampling gives with a 12-6 repulsion.
 *
 * Charges: exact counts of +1 and -1, the rest 0, placed by a seeded
 * Fisher-Yates shuffle.
 *
 * Velocities: Maxwell-Boltzmann at temperature T for mass m (Box-Muller),
 * then the mean velocity is removed so the net momentum is zero.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GEN_GAMMA 0x9E3779B97F4A7C15ULL
#define TAG_POS 0x504F534954494F4EULL /* "POSITION" */
#define TAG_CHG 0x4348415247455321ULL /* "CHARGES!" */
#define TAG_VEL 0x56454C4F43495459ULL /* "VELOCITY" */

static uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static uint64_t sm_out(uint64_t s, uint64_t n) { return mix64(s + (n + 1) * GEN_GAMMA); }

static double u53(uint64_t h) { return (double)(h >> 11) * 0x1.0p-53; }

/* Stream seed for (seed, tag, replica, particle). */
static uint64_t stream_key(uint64_t seed, uint64_t tag, uint64_t replica, uint64_t particle) {
  uint64_t k = sm_out(seed ^ tag, replica);
  return sm_out(k, particle);
}

/* --------------------------------------------------------------------- */
/* RSA positions                                                          */
/* --------------------------------------------------------------------- */

/* Returns 0 on success, -1 bad arguments, -2 out of memory, -3 too many
   rejections for some particle (density too high for d_min). */
int gen_rsa_positions(uint64_t seed, uint64_t replica, int64_t n, const double L[3], double dmin,
                      int64_t max_attempts, double *x, double *y, double *z) {
  if (n < 0 || !(L[0] > 0) || !(L[1] > 0) || !(L[2] > 0) || !(dmin >= 0)) return -1;
  if (n == 0) return 0;
  int nc[3];
  for (int d = 0; d < 3; ++d) {
    double e = dmin > 0 ? dmin : L[d];
    int c = (int)floor(L[d] / e);
    if (c < 1) c = 1;
    if (c > 2048) c = 2048;
    nc[d] = c;
  }
  int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
  int64_t *head = (int64_t *)malloc(sizeof(int64_t) * ncell);
  int64_t *next = (int64_t *)malloc(sizeof(int64_t) * n);
  if (!head || !next) { free(head); free(next); return -2; }
  for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
  const double d2min = dmin * dmin;
  /* with fewer than 3 cells along an axis the 27-cell scan would revisit
     cells; fall back to scanning every cell index once along that axis */
  int span[3];
  for (int d = 0; d < 3; ++d) span[d] = nc[d] >= 3 ? 1 : 0;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t key = stream_key(seed, TAG_POS, replica, (uint64_t)i);
    int placed = 0;
    for (int64_t a = 0; a < max_attempts && !placed; ++a) {
      double p[3];
      for (int d = 0; d < 3; ++d) {
        p[d] = L[d] * u53(sm_out(key, (uint64_t)(3 * a + d)));
        if (p[d] >= L[d]) p[d] = 0.0;
      }
      int c[3];
      for (int d = 0; d < 3; ++d) {
        c[d] = (int)(p[d] / L[d] * nc[d]);
        if (c[d] >= nc[d]) c[d] = nc[d] - 1;
      }
      int ok = 1;
      int lo[3], hi[3];
      for (int d = 0; d < 3; ++d) {
        if (span[d]) { lo[d] = c[d] - 1; hi[d] = c[d] + 1; }
        else { lo[d] = 0; hi[d] = nc[d] - 1; }
      }
      for (int cz = lo[2]; cz <= hi[2] && ok; ++cz)
        for (int cy = lo[1]; cy <= hi[1] && ok; ++cy)
          for (int cx = lo[0]; cx <= hi[0] && ok; ++cx) {
            int wx = (cx + nc[0]) % nc[0], wy = (cy + nc[1]) % nc[1], wz = (cz + nc[2]) % nc[2];
            for (int64_t j = head[((int64_t)wz * nc[1] + wy) * nc[0] + wx]; j >= 0; j = next[j]) {
              double dx = p[0] - x[j], dy = p[1] - y[j], dz = p[2] - z[j];
              dx -= L[0] * rint(dx / L[0]);
              dy -= L[1] * rint(dy / L[1]);
              dz -= L[2] * rint(dz / L[2]);
              if (dx * dx + dy * dy + dz * dz < d2min) { ok = 0; break; }
            }
          }
      if (ok) {
        x[i] = p[0]; y[i] = p[1]; z[i] = p[2];
        int64_t cell = ((int64_t)c[2] * nc[1] + c[1]) * nc[0] + c[0];
        next[i] = head[cell];
        head[cell] = i;
        placed = 1;
      }
    }
    if (!placed) { free(head); free(next); return -3; }
  }
  free(head);
  free(next);
  return 0;
}

/* --------------------------------------------------------------------- */
/* Charges                                                                */
/* --------------------------------------------------------------------- */

/* q[0..n): n_plus entries +qmag, n_minus entries -qmag, rest 0, shuffled. */
int gen_charges(uint64_t seed, uint64_t replica, int64_t n, int64_t n_plus, int64_t n_minus, double qmag,
                double *q) {
  if (n < 0 || n_plus < 0 || n_minus < 0 || n_plus + n_minus > n) return -1;
  for (int64_t i = 0; i < n; ++i) q[i] = i < n_plus ? qmag : (i < n_plus + n_minus ? -qmag : 0.0);
  uint64_t key = stream_key(seed, TAG_CHG, replica, 0);
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)(u53(sm_out(key, (uint64_t)i)) * (double)(i + 1));
    if (j > i) j = i;
    double t = q[i]; q[i] = q[j]; q[j] = t;
  }
  return 0;
}

/* --------------------------------------------------------------------- */
/* Velocities                                                             */
/* --------------------------------------------------------------------- */

int gen_velocities(uint64_t seed, uint64_t replica, int64_t n, double kT, double mass, double *vx, double *vy,
                   double *vz) {
  if (n < 0 || !(kT >= 0) || !(mass > 0)) return -1;
  if (n == 0) return 0;
  const double sd = sqrt(kT / mass);
  const double two_pi = 6.283185307179586476925286766559;
  double *v[3] = {vx, vy, vz};
  for (int64_t i = 0; i < n; ++i) {
    uint64_t key = stream_key(seed, TAG_VEL, replica, (uint64_t)i);
    for (int d = 0; d < 3; ++d) {
      double u1 = 1.0 - u53(sm_out(key, (uint64_t)(2 * d)));   /* (0, 1] */
      double u2 = u53(sm_out(key, (uint64_t)(2 * d + 1)));
      v[d][i] = sd * sqrt(-2.0 * log(u1)) * cos(two_pi * u2);
    }
  }
  for (int d = 0; d < 3; ++d) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += v[d][i];
    s /= (double)n;
    for (int64_t i = 0; i < n; ++i) v[d][i] -= s;
  }
  return 0;
}
