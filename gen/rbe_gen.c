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
 *
 * Large systems use the blocked RSA below (parallel, deterministic).
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
/* Blocked RSA for large systems                                          */
/* --------------------------------------------------------------------- */
/* The box is cut into an even number of blocks per axis (edge >= block_edge
   >= d_min), each block receiving floor(N/NB) or floor(N/NB)+1 particles
   (the first N mod NB blocks get one more). Blocks are filled colour by
   colour (8 colours by the parity of the block indices); blocks of one colour
   never touch, so they are filled in parallel, each by RSA inside the block
   against every particle already placed within d_min (own block and earlier
   colours). Every block draws from its own SplitMix64 stream, so the result
   does not depend on the thread count. Finally the particle order is
   shuffled (seeded Fisher-Yates) so that indices carry no spatial order. */
#define TAG_BLK 0x424C4F434B525341ULL /* "BLOCKRSA" */

int gen_rsa_blocked(uint64_t seed, uint64_t replica, int64_t n, const double L[3], double dmin, double block_edge,
                    int64_t max_attempts, double *x, double *y, double *z) {
  if (n < 0 || !(dmin > 0) || !(block_edge >= dmin)) return -1;
  for (int d = 0; d < 3; ++d)
    if (!(L[d] >= 2 * block_edge)) return -1;
  int nb[3], nf[3], kf[3];
  for (int d = 0; d < 3; ++d) {
    nb[d] = 2 * (int)floor(L[d] / (2.0 * block_edge));
    kf[d] = (int)floor(L[d] / nb[d] / dmin);
    if (kf[d] < 1) kf[d] = 1;
    nf[d] = nb[d] * kf[d];
  }
  const int64_t NB = (int64_t)nb[0] * nb[1] * nb[2];
  const int64_t NF = (int64_t)nf[0] * nf[1] * nf[2];
  int64_t *bstart = (int64_t *)malloc(sizeof(int64_t) * (NB + 1));
  int64_t *head = (int64_t *)malloc(sizeof(int64_t) * NF);
  int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
  double *px = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  double *py = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  double *pz = (double *)malloc(sizeof(double) * (n > 0 ? n : 1));
  if (!bstart || !head || !next || !px || !py || !pz) {
    free(bstart); free(head); free(next); free(px); free(py); free(pz);
    return -2;
  }
  const int64_t base = n / NB, extra = n % NB;
  bstart[0] = 0;
  for (int64_t b = 0; b < NB; ++b) bstart[b + 1] = bstart[b] + base + (b < extra ? 1 : 0);
  for (int64_t c = 0; c < NF; ++c) head[c] = -1;
  const double d2min = dmin * dmin;
  int failed = 0;
  for (int color = 0; color < 8; ++color) {
#pragma omp parallel for schedule(dynamic, 1) reduction(| : failed)
    for (int64_t b = 0; b < NB; ++b) {
      const int bx = (int)(b % nb[0]), by = (int)((b / nb[0]) % nb[1]), bz = (int)(b / ((int64_t)nb[0] * nb[1]));
      if ((bx & 1) + 2 * (by & 1) + 4 * (bz & 1) != color) continue;
      const int bc[3] = {bx, by, bz};
      uint64_t key = stream_key(seed, TAG_BLK, replica, (uint64_t)b);
      uint64_t draw = 0;
      for (int64_t i = bstart[b]; i < bstart[b + 1]; ++i) {
        int placed = 0;
        for (int64_t a = 0; a < max_attempts && !placed; ++a) {
          double p[3];
          int f[3];
          for (int d = 0; d < 3; ++d) {
            const double lo = L[d] * bc[d] / nb[d], hi = L[d] * (bc[d] + 1) / nb[d];
            p[d] = lo + (hi - lo) * u53(sm_out(key, draw++));
            if (p[d] >= hi) p[d] = lo;
            int fc = (int)(p[d] / L[d] * nf[d]);
            if (fc < bc[d] * kf[d]) fc = bc[d] * kf[d];
            if (fc > (bc[d] + 1) * kf[d] - 1) fc = (bc[d] + 1) * kf[d] - 1;
            f[d] = fc;
          }
          int ok = 1;
          for (int oz = -1; oz <= 1 && ok; ++oz)
            for (int oy = -1; oy <= 1 && ok; ++oy)
              for (int ox = -1; ox <= 1 && ok; ++ox) {
                const int wx = (f[0] + ox + nf[0]) % nf[0], wy = (f[1] + oy + nf[1]) % nf[1],
                          wz = (f[2] + oz + nf[2]) % nf[2];
                for (int64_t j = head[((int64_t)wz * nf[1] + wy) * nf[0] + wx]; j >= 0; j = next[j]) {
                  double dx = p[0] - px[j], dy = p[1] - py[j], dz = p[2] - pz[j];
                  dx -= L[0] * rint(dx / L[0]);
                  dy -= L[1] * rint(dy / L[1]);
                  dz -= L[2] * rint(dz / L[2]);
                  if (dx * dx + dy * dy + dz * dz < d2min) { ok = 0; break; }
                }
              }
          if (ok) {
            px[i] = p[0]; py[i] = p[1]; pz[i] = p[2];
            const int64_t cell = ((int64_t)f[2] * nf[1] + f[1]) * nf[0] + f[0];
            next[i] = head[cell];
            head[cell] = i;
            placed = 1;
          }
        }
        if (!placed) { failed = 1; break; }
      }
    }
    if (failed) break;
  }
  if (!failed) {
    /* seeded shuffle of the particle order */
    uint64_t skey = stream_key(seed, TAG_BLK, replica, (uint64_t)NB + 1);
    int64_t *perm = next; /* reuse */
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    for (int64_t i = n - 1; i > 0; --i) {
      int64_t j = (int64_t)(u53(sm_out(skey, (uint64_t)i)) * (double)(i + 1));
      if (j > i) j = i;
      int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int64_t i = 0; i < n; ++i) { x[i] = px[perm[i]]; y[i] = py[perm[i]]; z[i] = pz[perm[i]]; }
  }
  free(bstart); free(head); free(next); free(px); free(py); free(pz);
  return failed ? -3 : 0;
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
#pragma omp parallel for schedule(static)
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
