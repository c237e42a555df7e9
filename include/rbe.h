/*
 * rbe.h -- C ABI of the random batch Ewald (RBE) nonbonded force on one
 * AMD Instinct MI355X (gfx950).
 *
 * The library computes, for N point charges with Lennard-Jones cores in a
 * periodic box, the nonbonded force of RBMD 2.0 (arXiv 2609.02694, Sec. 2.1):
 *
 *   F_i = F_i^N + F_i^F
 *
 *   F_i^N  near field (Eq. 7-8): erfc-screened Coulomb within r_coul plus 12-6
 *          LJ (Eq. 2) within r_lj, over the minimum image, optionally through
 *          the core-shell random batch list (Eq. 10-11) with the momentum
 *          correction of Eq. 12;
 *   F_i^F  Fourier part by importance sampling (Eq. 9): P modes k_l drawn from
 *          P(k) ~ exp(-k^2/(4 alpha)) on the reciprocal lattice without k = 0,
 *          structure factors rho(k_l) = sum_j q_j exp(i k_l . r_j) (Eq. 5) and
 *          F_i^F = -kc q_i sum_l w_l k_l Im(exp(-i k_l . r_i) rho(k_l)),
 *          w_l = (S/P) 4 pi / (V k_l^2), S = sum_{k != 0} exp(-k^2/(4 alpha)).
 *
 * alpha is the paper's alpha: the real-space kernel is erfc(sqrt(alpha) r)/r
 * (Eq. 4). The sign convention is F = -grad U; pair terms act along
 * d = r_i - r_j.
 *
 * Conventions shared by every call
 *  - Pointers are DEVICE pointers unless marked (host).
 *  - `stream` is a hipStream_t passed as void*. rbe_forces, rbe_energy and
 *    rbe_step are asynchronous on it: they never wait for the device, so
 *    they can be captured in a HIP graph (with timing and counting off).
 *    Everything that depends on device data is decided on the device: the
 *    charged count that sizes the near-field and Fourier work is read there,
 *    and the neutrality of Eq. 1 and finite charges are checked there.
 *    rbe_sync_check synchronizes and reports device-side errors, among them
 *    RBE_ENONNEUTRAL and RBE_ENONFINITE; rbe_get_timing and rbe_get_counters
 *    synchronize to read their results.
 *  - Particle arrays are structure-of-arrays, FP64 for coordinates,
 *    velocities, forces and charges, int32 for ids.
 *  - Every call returns an rbe_status (0 = success). Host-checkable argument
 *    errors are rejected before any launch; rbe_last_error gives the message.
 *    No call aborts or throws across the ABI.
 *  - One context per stream at a time; a context is not thread-safe.
 */
#ifndef RBE_H
#define RBE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RBE_OK = 0,
  RBE_EINVAL = -1,      /* bad argument (sizes, cutoffs, null pointers)          */
  RBE_EBOX = -2,        /* a cutoff exceeds half the box (minimum image broken)  */
  RBE_ENONNEUTRAL = -3, /* sum q != 0 (Eq. 1 requires charge neutrality); checked
                           on the device, reported by rbe_sync_check            */
  RBE_ENOMEM = -4,      /* device allocation failed in rbe_create                */
  RBE_EDEVICE = -5,     /* a HIP call failed                                     */
  RBE_ENONFINITE = -6,  /* device saw a non-finite position/velocity/force       */
  RBE_ERANGE = -7       /* n exceeds the context capacity, or a bad particle id  */
} rbe_status;

typedef enum { RBE_FP64 = 0, RBE_FP32C = 1 } rbe_precision;

/* Fourier-mode distribution of the importance sample.
   RBE_KDIST_GAUSS: P(k) ~ exp(-k^2/(4 alpha)) (Eq. 9, the paper's), weights
     w = (S/P) 4 pi / (V k^2), S = sum_{k != 0} exp(-k^2/(4 alpha)).
   RBE_KDIST_GAUSS_OVER_K2: P(k) ~ exp(-k^2/(4 alpha))/k^2, weights
     w = (S2/P) 4 pi / V, S2 = sum_{k != 0} exp(-k^2/(4 alpha))/k^2 over the
     sampler's lattice; drawn by rejection from the Gaussian (acceptance
     k_min^2/k^2), so each draw costs more, the more so the larger the box.
     Not available in the batched form. */
typedef enum { RBE_KDIST_GAUSS = 0, RBE_KDIST_GAUSS_OVER_K2 = 1 } rbe_kdist;

/* Terms of F to evaluate (bit mask). */
enum { RBE_TERM_LJ = 1, RBE_TERM_COUL_REAL = 2, RBE_TERM_FOURIER = 4, RBE_TERM_ALL = 7 };

typedef struct {
  double L[3];        /* periodic box edges (Eq. 3)                                    */
  double alpha;       /* Ewald splitting parameter of Eq. 4 (> 0)                      */
  double r_coul;      /* real-space Coulomb cutoff: the paper's shell radius r_s       */
  double r_lj;        /* LJ cutoff (plain truncation)                                  */
  double r_core;      /* core radius r_c of Eq. 10; 0 disables the random batch list   */
  int32_t p_shell;    /* shell batch size p of Eq. 11 (1..32 when r_core > 0)          */
  int32_t P;          /* number of sampled Fourier modes (Eq. 9), 1..RBE_MAX_P         */
  int32_t kdist;      /* rbe_kdist                                                     */
  int32_t prec;       /* rbe_precision                                                 */
  int32_t terms;      /* RBE_TERM_* mask; 0 means RBE_TERM_ALL                         */
  int32_t ncell[3];   /* cell grid over the box (may differ per axis); 0 lets the
                         library choose: edge about max(r_lj, r_coul / 2) along y
                         and z, x cells four times finer                           */
  double lj_eps, lj_sigma; /* LJ parameters of Eq. 2                                   */
  double coulomb_k;   /* Coulomb prefactor kc (1 in reduced units); scales every
                         Coulomb term: real space, Fourier part and the energies      */
  double mass, dt;    /* particle mass and velocity-Verlet time step                   */
  double ghost_width; /* 0: periodic traversal; > 0: near field over a locally built
                         shell of periodic ghost copies of this width (>= r_coul)       */
  double nvt_kT;      /* Nose-Hoover target temperature k_B T (energy units)           */
  double nvt_tau;     /* Nose-Hoover relaxation time; 0: plain velocity Verlet (NVE).
                         > 0: rbe_step runs the NVT step below with thermostat mass
                         Q = N_f nvt_kT nvt_tau^2, N_f = 3N - 3                     */
  uint64_t seed;      /* stream seed of the mode sample and of the shell batches       */
  int32_t rbl_shell;  /* rbe_shell: population of the shell S_i of Eq. 10              */
} rbe_params;

/* Shell population of the random batch list. RBE_SHELL_ALL: every particle j
   with r_core < r <= r_coul (Eq. 10 as written). RBE_SHELL_CHARGED: the
   charged ones only (a variant: neutral shell members carry no force when
   r_lj <= r_core, which it requires, so the batch is spent on charges). */
enum { RBE_SHELL_ALL = 0, RBE_SHELL_CHARGED = 1 };

/* Sampled mode counts stay far below this; the bound is set by the full
   lattice of an exact Ewald reference run (rbe_lattice_modes). */
#define RBE_MAX_P 262144
#define RBE_MAX_SHELL_BATCH 32

/* Caller-owned particle state (device arrays of length n). The library never
   frees or reallocates them. fx, fy, fz receive forces; vx..vz and the
   positions are advanced by rbe_step. */
typedef struct {
  double *x, *y, *z;
  double *vx, *vy, *vz;
  double *fx, *fy, *fz;
  double *q;
  int32_t *id; /* unique, 0..n-1 (the shell batches of Eq. 11 are keyed by id) */
  double *nh;  /* NVT (nvt_tau > 0) only: device [2] = {xi, eta}, the thermostat's
                  friction variable and its time integral, advanced by rbe_step;
                  with forces that are the gradient of a potential U (fixed
                  modes, no batch list), K + U + Q xi^2/2 + N_f kT eta is
                  conserved up to the integrator's O(dt^2) error */
  int64_t n;
} rbe_state;

typedef struct rbe_ctx rbe_ctx;

/* Create a context for one system of up to n_max particles on HIP device
   `device` and allocate ALL its device scratch (cells, sorted copies, mode
   buffers, partial sums, flags). Validates *p (host): positive box, alpha,
   cutoffs <= L/2, 0 < P <= RBE_MAX_P, 1 <= p_shell <= 32 when r_core > 0,
   r_core <= r_coul, sqrt(alpha) r_coul <= 8, and with a ghost shell
   max(r_coul, r_lj) <= ghost_width <= L/2 and n_max < 2^28. On failure *out
   is NULL and the status says why. */
int rbe_create(rbe_ctx **out, const rbe_params *p /* host */, int64_t n_max, int device);

/* Batched form: n_sys independent systems ("replicas"), replica s owning
   particles [offset[s], offset[s+1]) of every state array (offset[0] = 0,
   each replica at least one particle, offset[n_sys] < 2^31). params[s]
   gives replica s its box L, cell grid ncell and stream seed; every other
   field must be the same in all entries. The random batch list (r_core > 0)
   and the ghost shell (ghost_width > 0) are not available in this form.
   Each replica is an independent periodic system: its own cells, its own
   mode sample of Eq. 9 (drawn from its own seed for the common eval) and its
   own structure factors. rbe_forces and rbe_step then take the concatenated
   state (n = offset[n_sys]); rbe_forces requires m, w and rho_out to be NULL.
   rbe_step runs every velocity-Verlet step of all replicas in three launches
   (a persistent kernel for binning and reorder, a near-field kernel, the
   persistent kernel again for the Fourier part and the second half-kick;
   captured two steps at a time in a HIP graph) and returns each
   replica's particles in cell order inside its own range. rbe_build_cells is
   not available on a batched context. With n_sys == 1 this is rbe_create
   with n_max = offset[1] - offset[0]. */
int rbe_create_batch(rbe_ctx **out, int32_t n_sys, const rbe_params *params /* host */,
                     const int64_t *offset /* host */, int device);

void rbe_destroy(rbe_ctx *ctx);

/* Message of the last failed call on ctx (or of the last failed create when
   ctx is NULL). Never NULL. */
const char *rbe_last_error(const rbe_ctx *ctx);

/* Cell binning (Sec. 2.2: linked cells with cell-wise reordering).
   key_i = s_i * C + (c_z * n_y + c_y) * n_x + c_x, with s_i = 0 for charged and
   1 for neutral particles, C = n_x n_y n_z, and
   c_d = min(n_d - 1, floor(w_d * (n_d / L_d))), w the coordinate wrapped into
   [0, L_d). Output: the stable counting sort of the particles by key
   (ties in input order): perm[0..n) lists input indices in key order and
   cell_start[0..2C] holds the first slot of every key (cell_start[2C] = n).
   Bit-exact: the result is a pure function of the inputs. */
int rbe_build_cells(rbe_ctx *ctx, const double *x, const double *y, const double *z, const double *q, int64_t n,
                    int32_t *cell_start, int32_t *perm, void *stream);

/* Importance sample of Eq. 9 for force evaluation `eval`: writes m[3*P]
   (integer mode vectors, blocks x | y | z, k = 2 pi m / L) and w[P] (the
   weights of p->kdist). Draw l, attempt a uses outputs 3a..3a+2 of a
   SplitMix64 stream keyed by (seed, eval, l); each output is mapped through
   the per-axis inverse CDF of exp(-(pi m / L_d)^2 / alpha) and m = 0 is
   rejected. RBE_KDIST_GAUSS_OVER_K2: attempt a uses outputs 4a..4a+2 that
   way and is accepted when m != 0 and u k^2 < k_min^2 with u = output 4a+3
   and k_min = 2 pi / max_d L_d. on_device = 0: m, w are HOST pointers, computed on the host;
   on_device = 1: DEVICE pointers, computed by a kernel on `stream`. Both
   paths give identical bits. */
int rbe_sample_k(const rbe_params *p /* host */, uint64_t eval, int32_t *m, double *w, int on_device,
                 void *stream);

/* The Ewald reciprocal sum (Eq. 5 with every lattice mode, Sec. 2.1) as a
   mode table: the modes 0 < |k| <= k_max, k = 2 pi (m_x/L_x, m_y/L_y, m_z/L_z),
   of the half space (m_x > 0, or m_x = 0 and m_y > 0, or m_x = m_y = 0 and
   m_z > 0), each standing for itself and -k, with weight
   w = 2 * 4 pi exp(-k^2/(4 alpha)) / (V k^2). Given to rbe_forces,
   rbe_energy or rbe_set_modes on a context with P = the count, the Fourier
   part is the deterministic Ewald sum truncated at k_max instead of the
   importance sample of Eq. 9 (a reference for accuracy checks; its cost
   grows as k_max^3 V). Host function: reads p->L and p->alpha only.
   m == NULL: only *count is set. Otherwise m (host, 3 rows of cap entries:
   m_x, then m_y, then m_z) and w (host, cap entries) are filled, cap must
   equal the count (RBE_ERANGE otherwise), in the order of increasing m_x,
   then m_y, then m_z. RBE_ERANGE also when k_max spans more than 4096 modes
   along an axis. */
int rbe_lattice_modes(const rbe_params *p /* host */, double k_max, int32_t *m /* host */, double *w /* host */,
                      int32_t cap, int32_t *count /* host */);

/* Fixes the mode table of a single-system context: from this call on,
   rbe_forces and rbe_energy with m == NULL and every step of rbe_step use
   (m, w) (device, 3*P and P entries as rbe_sample_k lays them out; copied
   on `stream`, so the caller may free them after the stream has run)
   instead of drawing the sample of each evaluation. With the table of
   rbe_lattice_modes and r_core = 0 the dynamics is plain Ewald molecular
   dynamics, the reference the random batch estimates are compared with.
   m == w == NULL returns to drawing. RBE_EINVAL on a batched context. */
int rbe_set_modes(rbe_ctx *ctx, const int32_t *m, const double *w, void *stream);

/* One force evaluation F = F^N + F^F on the state as given (never reorders
   it): writes s->fx, fy, fz in the caller's particle order. (m, w) is the
   mode sample (device, 3*P and P entries); if m is NULL the library draws it
   for `eval` itself. eval also keys the shell batches of Eq. 11.
   rho_out, if not NULL, receives Re rho | Im rho (2*P doubles, device). */
int rbe_forces(rbe_ctx *ctx, const rbe_state *s, const int32_t *m, const double *w, uint64_t eval,
               double *rho_out, void *stream);

/* Energy and virial terms of Sec. 2.1 for the state as given (diagnostics:
   energy conservation, pressure), computed in FP64 whatever the context's
   precision, into u_out[0..RBE_ENERGY_TERMS) (device doubles):
     [RBE_U_COUL_REAL] kc sum_{i<j} q_i q_j erfc(sqrt(alpha) r)/r over every
                       pair with r <= r_coul (minimum image): the screened
                       part of Eq. 4, the energy whose gradient is the near
                       field of Eq. 7-8. The random batch list of Eq. 10-11
                       is a force estimator only: every pair inside the
                       cutoff is counted here;
     [RBE_U_LJ]        sum_{i<j} 4 eps ((sigma/r)^12 - (sigma/r)^6) over
                       r <= r_lj (Eq. 2, plain truncation, no shift);
     [RBE_U_FOURIER]   kc (1/2) sum_l w_l |rho(k_l)|^2 = kc (S/P)(2 pi/V)
                       sum_l |rho(k_l)|^2 / k_l^2: the importance-sampling
                       estimate of Eq. 5 with the modes of Eq. 9. (m, w) is
                       the mode sample (device); m NULL draws the one of
                       `eval`, the same as rbe_forces and rbe_sample_k;
     [RBE_U_SELF]      kc sqrt(alpha/pi) sum_i q_i^2 (Eq. 6);
     [RBE_U_KINETIC]   (mass/2) sum_i |v_i|^2, 0 when s->vx..vz are NULL;
     [RBE_W_COUL_REAL] sum_{i<j} d_ij . F_ij of the screened Coulomb pairs:
                       kc q_i q_j r^2 G(r) with G of Eq. 8;
     [RBE_W_LJ]        sum_{i<j} r^2 G_LJ(r) (Eq. 8);
     [RBE_W_FOURIER]   kc (1/2) sum_l w_l |rho(k_l)|^2 (1 - k_l^2/(2 alpha)):
                       minus the derivative of U_FOURIER under a uniform
                       dilation of positions and box.
   The potential energy is U_COUL_REAL + U_LJ + U_FOURIER - U_SELF, and the
   pressure (2 U_KINETIC + W_COUL_REAL + W_LJ + W_FOURIER) / (3 V) (the self
   energy does not depend on the volume). Terms left out of the context's
   `terms` mask are 0 (U_SELF goes with the Fourier term). Only s->x, y, z, q (and v when given) are read; f and id
   may be NULL. rho_out as in rbe_forces. Not available on a batched
   context. */
enum { RBE_U_COUL_REAL = 0, RBE_U_LJ = 1, RBE_U_FOURIER = 2, RBE_U_SELF = 3, RBE_U_KINETIC = 4,
       RBE_W_COUL_REAL = 5, RBE_W_LJ = 6, RBE_W_FOURIER = 7, RBE_ENERGY_TERMS = 8 };
int rbe_energy(rbe_ctx *ctx, const rbe_state *s, const int32_t *m, const double *w, uint64_t eval,
               double *u_out, double *rho_out, void *stream);

/* nsteps velocity-Verlet steps:
     v += dt/(2m) F;  x <- wrap(x + dt v);  F <- force(x, eval = first_eval + k);
     v += dt/(2m) F
   for k = 0..nsteps-1. On entry s->f* must hold the force of the current
   positions. Positions, velocities, forces, charges and ids are returned in
   cell order (the particles are reordered; id[] maps them back).
   NVT (nvt_tau > 0; the paper runs every experiment in the Nose-Hoover
   canonical ensemble, Sec. 3): each step is wrapped in two half-steps of a
   single Nose-Hoover thermostat (symmetric Trotter split), with
   K = (m/2) sum |v|^2 and G(K) = (2K - N_f kT)/Q:
     half: xi += dt/4 G(K); v *= exp(-xi dt/2); eta += xi dt/2; xi += dt/4 G(K)
     step: half; v += dt/(2m) F; x <- wrap(x + dt v); F <- force; v += dt/(2m) F; half
   s->nh must then point to {xi, eta} on the device; n >= 2. Not available on
   a batched context. */
int rbe_step(rbe_ctx *ctx, rbe_state *s, int32_t nsteps, uint64_t first_eval, void *stream);

/* rbe_forces for callers that cannot allocate device memory (code under HIP
   graph capture, tight serving loops, harnesses that forbid hipMalloc): no
   context, no hipMalloc or hipFree, no allocating library call. The scratch
   lives in one file-scope device array of RBE_NOALLOC_SCRATCH_BYTES per GPU
   (held until the process ends), shared by every call on that GPU: calls that
   overlap on one GPU race, so serialize them (one stream, or events).
   Computes the same force as rbe_forces on a context created with *p, on the
   current HIP device, for the state as given (never reordered): writes
   s->fx, fy, fz; rho_out (device, 2*P doubles) may be NULL.
   Limits, rejected with RBE_ERANGE before any launch: n <= RBE_NOALLOC_MAX_N,
   P <= RBE_NOALLOC_MAX_P, 2 * (cells of the grid) <= RBE_NOALLOC_MAX_KEYS; the
   ghost shell is not available (RBE_EINVAL). m and w (the mode sample,
   device) are required. Device-side checks (neutrality, finite values, ids)
   are not kept for a later rbe_sync_check: status_out (device int32, may be
   NULL) receives the rbe_status they give once the stream reaches the end of
   the call. Host errors are reported by rbe_last_error(NULL). */
#define RBE_NOALLOC_MAX_N 32768
#define RBE_NOALLOC_MAX_P 1024
#define RBE_NOALLOC_MAX_KEYS 131072
#define RBE_NOALLOC_SCRATCH_BYTES (8 << 20)
int rbe_forces_noalloc(const rbe_params *p /* host */, const rbe_state *s, const int32_t *m, const double *w,
                       uint64_t eval, double *rho_out, int32_t *status_out, void *stream);

/* Synchronize `stream` and report device-side errors recorded since the last
   check: non-neutral charges (RBE_ENONNEUTRAL; a batched context names the
   first replica at fault), non-finite charges, velocities or forces
   (RBE_ENONFINITE), bad ids and ghost-shell overflow (RBE_ERANGE), a mode
   sampler that rejected every attempt (RBE_EINVAL). Clears the flag. The
   only call that waits for the device, besides the timing and counter
   readers. */
int rbe_sync_check(rbe_ctx *ctx, void *stream);

/* Diagnostic counters of the last rbe_forces/rbe_step force evaluation
   (host, 12 entries = 3 near-field parts x 4): part k in {0: charged
   particles (plain sums, or core and shell of the random batch list),
   1: reserved (zero), 2: neutral particles}; entry [4k + 0] Coulomb pair
   terms evaluated (both
   charged, inside the cutoff), [4k + 1] LJ pair terms evaluated (inside
   r_lj), [4k + 2] candidate pairs tested, [4k + 3] shell members ranked
   (sum of #S_i, Eq. 10).
   Only filled when counting was enabled with rbe_set_counting(ctx, 1); the
   counting adds atomics to the near-field kernel and is meant for the
   roofline figures, not for timed runs. */
int rbe_set_counting(rbe_ctx *ctx, int enable);
int rbe_get_counters(rbe_ctx *ctx, int64_t *counters /* host, 12 */, void *stream);

/* Per-kernel timing with HIP events recorded on the call's stream around
   every launch of the kinds below (enable = 1 starts and clears the
   accumulation; 0 stops it). rbe_get_timing synchronizes `stream`, then
   writes, per kind, the summed duration in ms (ms_out) and the launch count
   (launches_out), host arrays of RBE_TIMING_KINDS entries. */
enum {
  RBE_TK_BIN = 0,         /* keys, histogram, scan, stable placement        */
  RBE_TK_REORDER = 1,     /* reorder + packing of the sorted records        */
  RBE_TK_PAIR = 2,        /* near field of the neutral particles            */
  RBE_TK_MEAN = 3,        /* Eq. 12 mean                                    */
  RBE_TK_SAMPLE = 4,      /* device mode sampler + mode conversion          */
  RBE_TK_RHO_PARTIAL = 5, /* structure-factor chunk partials                */
  RBE_TK_RHO_FINAL = 6,   /* fixed-order final sum                          */
  RBE_TK_GATHER = 7,      /* Fourier force gather                           */
  RBE_TK_KICK_DRIFT = 8,  /* first half-kick + drift + wrap (from a call's
                             second step on, fused with the previous step's
                             second half-kick)                              */
  RBE_TK_KICK = 9,        /* second half-kick (+ mean subtraction) of a
                             call's last step; with NVT, every step's second
                             half-kick with the kinetic-energy sum and the
                             thermostat half-steps                          */
  RBE_TK_PAIR_CHARGED = 10, /* near field of the charged particles (core)   */
  RBE_TK_PAIR_SHELL = 11, /* reserved: the shell of Eq. 11 is timed with
                             RBE_TK_PAIR_CHARGED (one fused launch)          */
  RBE_TK_GHOST = 12,      /* ghost shell build and sort                     */
  RBE_TK_BATCH = 13,      /* step of a batched context (one entry per step,
                             its three launches together)                   */
  RBE_TIMING_KINDS = 14
};
int rbe_set_timing(rbe_ctx *ctx, int enable);
int rbe_get_timing(rbe_ctx *ctx, double *ms_out /* host */, int64_t *launches_out /* host */, void *stream);

#ifdef __cplusplus
}
#endif
#endif
