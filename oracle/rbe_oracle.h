/*
 * rbe_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference for the random batch Ewald (RBE) nonbonded
 * force of RBMD 2.0 (arXiv 2609.02694). Only the test-suite, the smoke check
 * and the CPU-baseline leg of the benchmark may call it. It shares no code
 * with the GPU library.
 *
 * Units: the Coulomb prefactor is an argument (1 in reduced LJ units);
 * alpha is the paper's alpha, i.e. the real-space kernel is erfc(sqrt(alpha) r)/r
 * (Sec. 2.1, Eq. 4).
 */
#ifndef RBE_ORACLE_H
#define RBE_ORACLE_H
#include <stdint.h>

typedef struct {
  double L[3];      /* periodic box */
  double alpha;     /* Ewald splitting parameter of Eq. 4 */
  double r_coul;    /* real-space Coulomb cutoff (the paper's shell radius r_s) */
  double r_lj;      /* Lennard-Jones cutoff (plain truncation) */
  double r_core;    /* core radius of the random batch list; 0 disables the list */
  int32_t p_shell;  /* shell batch size p of Eq. 11 */
  double eps, sigma;/* LJ parameters of Eq. 2 (one species pair) */
  double kc;        /* Coulomb prefactor */
  int32_t shell_charged; /* 1: the shell of Eq. 10 holds charged particles only
                            (variant; needs r_lj <= r_core), 0: every particle */
} orc_sys;

/* term selection bits */
#define ORC_LJ 1
#define ORC_COUL_REAL 2
#define ORC_FOURIER 4

/* SplitMix64 helpers exposed for tests */
uint64_t orc_mix64(uint64_t z);
uint32_t orc_rbl_key(uint64_t seed, uint64_t eval, int32_t id_i, int32_t id_j);

/* --- Fourier-mode sampling (Sec. 2.1, Eq. 9) --- */
int orc_axis_cutoff(double L, double alpha);
double orc_axis_H(double L, double alpha);
double orc_norm_S(const double L[3], double alpha);
/* kdist 0: P(k) ~ exp(-k^2/4a) (Eq. 9).  Writes m[3*P] (x block, y block, z
   block) and w[P]. Returns 0 or a negative status. */
/* normalizer of the exp(-k^2/4a)/k^2 proposal over the sampler's lattice */
double orc_norm_S2(const double L[3], double alpha);
int orc_sample_k(uint64_t seed, uint64_t eval, const double L[3], double alpha, int32_t P, int32_t kdist,
                 int32_t *m, double *w);

/* --- structure factor and Fourier force for a given mode set (Eq. 5, 7, 9) --- */
void orc_rho(int64_t n, const double *x, const double *y, const double *z, const double *q, const double L[3],
             int32_t P, const int32_t *m, double *rho_re, double *rho_im);
void orc_fourier_force(int64_t n, const double *x, const double *y, const double *z, const double *q,
                       const double L[3], int32_t P, const int32_t *m, const double *w, const double *rho_re,
                       const double *rho_im, double *fx, double *fy, double *fz);
/* U* = 1/2 sum_l w_l |rho_l|^2 : the energy whose exact gradient is the fixed-mode force */
double orc_fourier_energy(int32_t P, const double *w, const double *rho_re, const double *rho_im);
/* W* = 1/2 sum_l w_l |rho_l|^2 (1 - k_l^2/(2 alpha)) : minus the dilation derivative of U* */
double orc_fourier_virial(int32_t P, const int32_t *m, const double L[3], double alpha, const double *w,
                          const double *rho_re, const double *rho_im);

/* --- real space (Eq. 2, 7, 8, 10-12) --- */
/* Full-list near-field force on the particles listed in idx[0..nidx) (all if
   idx == NULL), brute force over every j with the minimum image. With
   r_core > 0 the random batch list of Eq. 11 is applied (no Eq. 12 mean). */
void orc_real_force(int64_t n, const double *x, const double *y, const double *z, const double *q,
                    const int32_t *id, const orc_sys *s, int32_t terms, uint64_t seed, uint64_t eval,
                    int64_t nidx, const int64_t *idx, double *fx, double *fy, double *fz, int64_t *n_shell);
/* Same result computed through a cell grid (faster for large n); every i. */
int orc_real_force_cells(int64_t n, const double *x, const double *y, const double *z, const double *q,
                         const int32_t *id, const orc_sys *s, int32_t terms, uint64_t seed, uint64_t eval,
                         int64_t nidx, const int64_t *idx, double *fx, double *fy, double *fz);
/* Eq. 12: subtract the mean over all n particles. */
void orc_mean_correct(int64_t n, double *fx, double *fy, double *fz, double mean_out[3]);
/* real-space energies (i<j) over minimum images within the cutoffs */
void orc_real_energy(int64_t n, const double *x, const double *y, const double *z, const double *q,
                     const orc_sys *s, double *u_coul, double *u_lj);

/* real-space pair virials sum_{i<j} d_ij . F_ij within the cutoffs */
void orc_real_virial(int64_t n, const double *x, const double *y, const double *z, const double *q,
                     const orc_sys *s, double *w_coul, double *w_lj);

/* --- exact Ewald sum for tiny boxes (Eq. 3-8) --- */
void orc_ewald_exact(int64_t n, const double *x, const double *y, const double *z, const double *q,
                     const double L[3], double alpha, double tol, double *u_real, double *u_recip, double *u_self,
                     double *fx, double *fy, double *fz);
/* Self energy of Eq. 6 (without a Coulomb prefactor) and the kinetic energy. */
double orc_self_energy(int64_t n, const double *q, double alpha);
double orc_kinetic_energy(int64_t n, const double *vx, const double *vy, const double *vz, double mass);
/* Deterministic full-lattice mode set with weights 4 pi exp(-k^2/4a)/(V k^2),
   all m != 0 with |m_d| <= mmax[d]. Returns the mode count (m, w may be NULL
   to query it). */
int64_t orc_full_lattice(const double L[3], double alpha, const int32_t mmax[3], int32_t *m, double *w);

/* --- cell binning: stable counting sort by (species, cell) --- */
int orc_bin(int64_t n, const double *x, const double *y, const double *z, const double *q, const double L[3],
            const int32_t ncell[3], int32_t *cell_start, int32_t *perm);

/* --- one velocity-Verlet step (positions wrapped into [0, L)) --- */
void orc_kick(int64_t n, double half_dt_over_m, const double *fx, const double *fy, const double *fz, double *vx,
              double *vy, double *vz);
void orc_drift_wrap(int64_t n, double dt, const double L[3], const double *vx, const double *vy, const double *vz,
                    double *x, double *y, double *z);

int orc_num_threads(void);
void orc_set_num_threads(int k);
#endif
