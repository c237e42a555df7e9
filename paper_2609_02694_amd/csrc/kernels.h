// Kernel launchers of the RBE library (internal).
#pragma once
#include "rbe_internal.h"

namespace rbe {

// ---------------------------------------------------------------------------
// binning
// ---------------------------------------------------------------------------
struct BinBuffers {
  int32_t *key;       // [n_max]
  int32_t *slot;      // [n_max]
  int32_t *count;     // [2 * ncell]
  int32_t *tmp;       // [n_max]
  int32_t *scan_tmp;  // [scan_tiles(2 * ncell)]
};
int64_t scan_tiles(int64_t n);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t st);
void launch_fill_f64(double *p, int64_t n, double v, hipStream_t st);
void launch_exclusive_scan(const int32_t *cnt, int64_t n, int32_t *start, int32_t *tmp, hipStream_t st);
void launch_bin(const BinBuffers &b, const Grid &g, int64_t n, const double *x, const double *y, const double *z,
                const double *q, int32_t *cell_start, int32_t *perm, hipStream_t st);
// The passes of launch_bin around its keys pass, for a keys pass fused into
// another kernel: clearing the histogram, then scan, scatter and placement.
void launch_bin_clear(const BinBuffers &b, const Grid &g, hipStream_t st);
void launch_bin_place(const BinBuffers &b, const Grid &g, int64_t n, int32_t *cell_start, int32_t *perm,
                      hipStream_t st);

// ---------------------------------------------------------------------------
// sorted working copies
// ---------------------------------------------------------------------------
// Packed per-particle records in cell order:
//   xq[i] = (x, y, z, q) wrapped coordinates (near field)
//   sq[i] = (x/L_x, y/L_y, z/L_z, q) fractional coordinates (Fourier part,
//           only the charged range [0, nq) is used)
struct Sorted {
  double4 *xq;
  double4 *sq;
  int32_t *id;
};
// Gather the caller's arrays through perm into the packed sorted records
// (id may be nullptr: then s.id is left as it is).
void launch_gather_sorted(int64_t n, const int32_t *perm, const double *x, const double *y, const double *z,
                          const double *q, const int32_t *id, const Grid &g, Sorted s, hipStream_t st);
// Build the inverse id map inv[id[k]] = k (flags ids outside [0, n)).
void launch_inverse_ids(int64_t n, const int32_t *id_sorted, int32_t *inv, int *err, hipStream_t st);
// out[perm[k]] = in[k] for the three force components.
void launch_scatter_forces(int64_t n, const int32_t *perm, const double *fx, const double *fy, const double *fz,
                           double *ox, double *oy, double *oz, hipStream_t st);

// ---------------------------------------------------------------------------
// ghost shell (ghost_width > 0)
// ---------------------------------------------------------------------------
struct GhostBuffers {
  int64_t cap;             // ghost capacity
  double4 *xq;             // [cap + kScanPad] ghost records in padded cell order
  int32_t *id;             // [cap + kScanPad] ids of their natives
  int32_t *cell_start;     // [2 * pncell + 1] first ghost of every padded key (clamped to cap)
  int32_t *cell_count;     // [2 * pncell]
  int32_t *cell_scan_tmp;  // [scan_tiles(2 * pncell)]
  int32_t *count;          // [1] ghosts made (device)
};
// Builds the ghost shell of the sorted natives s[0..n) (cell_start: their
// cell table) in padded cell order.
void launch_build_ghosts(const Grid &g, int64_t n, const int32_t *cell_start, const Sorted &s,
                         const GhostBuffers &gb, int *err, hipStream_t st);

// ---------------------------------------------------------------------------
// near field
// ---------------------------------------------------------------------------
// Stencil radius in cells along each axis (grids may be finer along x, where
// each stencil row is trimmed per particle, than along y and z).
struct Sten {
  int x, y, z;
};
struct PairParams {
  Grid g;
  Sten s_coul;           // stencil radii covering max(r_coul, r_lj)
  Sten s_lj;             // stencil radii covering r_lj
  Sten s_core;           // stencil radii covering max(r_core, r_lj)
  double rc2, rlj2, rcore2;
  double rq2;            // max(rc2, rlj2): reach of a charged pair
  double alpha, sqrt_alpha, two_sqrt_alpha_over_sqrt_pi;
  double kc, eps24, sig2;
  int do_coul, do_lj;
  int rbl;               // random batch list on
  int shell_charged;     // shell of charged particles only (variant; r_lj <= r_core)
  int p_shell;
  uint64_t shell_key;    // stream key of the shell batches for this evaluation
  uint64_t shell_T0;     // first key threshold of the shell selection (<= 2^32)
};
// FP32 copies of the pair constants (FP32C form).
struct PairF32 {
  float sqrt_alpha, neg_alpha_log2e, two_sqrt_alpha_over_sqrt_pi, kc, eps24, sig2;
};
PairF32 make_pair_f32(const PairParams &pp);
// Shell selection of the random batch list: keys collected per particle, and
// the first threshold (about 3p keys below it for the mean shell of n
// particles in the box; 2^32 = all keys when shells are small).
constexpr int kShellCap = 128;
// Records of padding after every particle array a thread-form neighbour
// scan reads (sorted natives, ghosts, batch): its lookahead loads may run
// up to this many records minus one past the end of a range.
constexpr int kScanPad = 8;
__host__ __device__ inline uint64_t shell_first_threshold(const PairParams &pp, int64_t n) {
  const double V = pp.g.L[0] * pp.g.L[1] * pp.g.L[2];
  const double rc = sqrt(pp.rc2), r0 = sqrt(pp.rcore2);
  const double m_mean = (double)n / V * (4.0 / 3.0) * kPi * (rc * rc * rc - r0 * r0 * r0);
  if (!(m_mean > 0.5 * kShellCap)) return 1ull << 32;
  const double f = 3.0 * pp.p_shell / m_mean;
  if (f >= 1.0) return 1ull << 32;
  return (uint64_t)(f * 4294967296.0);
}
struct PairCounters {
  unsigned long long *c;  // [4] or nullptr
};
// Near-field force; charged particles are [0, nq) of the sorted order,
// neutral ones [nq, n), with nq read on the device (*nq). Launched in two
// parts: charged particles (plain sums, or core and shell of the random batch
// list) and neutral particles.
// PAIR_PART_SHELL launches nothing (kept for the counter layout).
// PAIR_PART_COULOMB: the charged particles' screened Coulomb terms only,
// added to f (which holds their LJ terms from launch_lj_tile).
enum { PAIR_PART_CHARGED = 0, PAIR_PART_SHELL = 1, PAIR_PART_NEUTRAL = 2, PAIR_PART_COULOMB = 3 };
// gb: ghost shell of the natives (nullptr for the periodic traversal).
void launch_pair(int prec, int part, const PairParams &pp, int64_t n, const int32_t *nq, const Sorted &s,
                 const int32_t *cell_start, const int32_t *inv_id, const GhostBuffers *gb, double *fx, double *fy,
                 double *fz, PairCounters cnt, hipStream_t st);

// LJ terms of every particle of the species blocks in iblk (bit 0 charged,
// bit 1 neutral) over LDS-staged cell tiles, FP32C form: writes f of those
// particles (counters [4] or nullptr: [1] LJ pair terms, [2] candidates).
// Used on grids whose mean cell occupancy suits the staging
// (lj_tile_applicable, false for every other precision); the other cases
// keep the thread-form walks.
bool lj_tile_applicable(int prec, const PairParams &pp, int64_t n);
void launch_lj_tile(const PairParams &pp, int64_t n, int iblk, const Sorted &s, const int32_t *cell_start,
                    const GhostBuffers *gb, double *fx, double *fy, double *fz, unsigned long long *counters,
                    int *err, hipStream_t st);

// ---------------------------------------------------------------------------
// Fourier part
// ---------------------------------------------------------------------------
struct GatherMode {
  double mx, my, mz;                // integer mode vector as doubles
  double a, b;                      // w Im rho, w Re rho
  float af, bf, mxf, myf, mzf, pad; // FP32 copies for the FP32C gather
};
struct FourierBuffers {
  double *mkd;           // [3][P] mode vectors as doubles
  double2 *part;         // [nchunk_max][P] partial structure factors
  double *rho;           // [2 * P] Re | Im
  GatherMode *modes;     // [P]
  double2 *turn_tab;     // [kTurnTableEntries] (sin, cos) of 2 pi k / kTurnTableEntries (FP64 kernels)
  double4 *gpart;        // [kGatherPartMax] per-group gather sums (mode split); nullptr: no split
  int nchunk_max;
};
// Entries of the gather's per-group partial sums: the mode split is used only
// while groups x (charged range rounded to blocks) fits.
constexpr int64_t kGatherPartMax = 262144;
constexpr int kTurnTableEntries = 256;
// Host values of the FP64 kernels' turn table (n entries of (sin, cos) of
// 2 pi k / n, each rounded once from extended precision).
void fill_turn_table(double2 *host, int n);
// Chunk layout of the structure-factor partial sums of nq charged particles:
// enough chunks to fill the chip (about 8k waves), chunks of at least 64
// particles, never more chunks than the scratch holds. Returns the chunk
// length; *nchunks receives the chunk count (at least 1). Evaluated on the
// device from the device-side count, so the launches need no host copy of nq.
__host__ __device__ inline int rho_layout(int64_t nq, int P, int nchunk_max, int *nchunks) {
  const int64_t groups = (P + 63) / 64;
  const int64_t target = (8192 + groups - 1) / groups;
  int64_t len = (nq + target - 1) / target;
  if (len < 64) len = 64;
  while ((nq + len - 1) / len > nchunk_max) len *= 2;
  const int64_t nc = (nq + len - 1) / len;
  *nchunks = nc < 1 ? 1 : (int)nc;
  return (int)len;
}
// Upper bound of rho_layout's chunk count over every nq <= nq_max (the grid
// of the partial-sum launch; blocks past the actual count exit at once).
inline int rho_max_chunks(int64_t nq_max, int P, int nchunk_max) {
  const int64_t groups = (P + 63) / 64;
  int64_t m = (8192 + groups - 1) / groups;
  if (m > nchunk_max) m = nchunk_max;
  const int64_t by_len = (nq_max + 63) / 64;
  if (m > by_len) m = by_len;
  return m < 1 ? 1 : (int)m;
}
void launch_modes_to_double(int P, const int32_t *m, double *mkd, hipStream_t st);
// The charged count nq is read on the device (*nq, the first neutral cell
// start); nq_max bounds it (sizes the grids).
void launch_rho_partial(int prec, const int32_t *nq, int64_t nq_max, int P, const double4 *sq,
                        const FourierBuffers &fb, hipStream_t st);
// The gather coefficients take the weights times kc (the Coulomb prefactor
// scales the Fourier force like every other Coulomb term).
void launch_rho_final(const int32_t *nq, int P, const FourierBuffers &fb, const double *w, double kc,
                      double *rho_out, hipStream_t st);
void launch_fourier_gather(int prec, const int32_t *nq, int64_t nq_max, int P, const double4 *sq,
                           const FourierBuffers &fb, const Grid &g, double *fx, double *fy, double *fz,
                           hipStream_t st);

// ---------------------------------------------------------------------------
// energy terms (diagnostics, FP64)
// ---------------------------------------------------------------------------
struct EnergyFinal {
  const double *near_part;  // [4 nb_near] block partials (Coulomb and LJ energy, Coulomb and LJ
                            // virial); set by launch_energy
  int64_t nb_near;
  const double *sq_part;    // [2 nb_sq] block partials (q^2, |v|^2); set by launch_energy
  int64_t nb_sq;
  const double *w, *rho;    // mode weights [P] and Re | Im rho [2 P]; rho nullptr: no Fourier term
  const double *mkd;        // [3][P] mode vectors as doubles
  int P;
  double L[3], alpha;
  double kc, self_coef, half_mass;  // kc, kc sqrt(alpha/pi), mass/2
  double *out;              // [8] device
};
// Length of the partial-sum scratch launch_energy needs for n_max particles.
int energy_part_len(int64_t n_max);
// Near-field energies of the sorted particles (when near), the q^2 and v^2
// sums of the caller's arrays (vx may be nullptr), and the final fixed-order
// combination into fin.out.
void launch_energy(const PairParams &pp, double lj4, int64_t n, const Sorted &s,
                   const int32_t *cell_start, bool near, const double *q, const double *vx, const double *vy,
                   const double *vz, double *part, EnergyFinal fin, hipStream_t st);

// ---------------------------------------------------------------------------
// reductions and integration
// ---------------------------------------------------------------------------
// mean[3] = (1/n) sum_i f_i in a fixed order (partials[nblk * 3] scratch).
int mean_blocks(int64_t n);
void launch_mean3(int64_t n, const double *fx, const double *fy, const double *fz, double *partials, double *mean,
                  hipStream_t st);
// f -= mean (if mean != nullptr); v += h f; flags non-finite f or v.
void launch_kick(int64_t n, double h, const double *mean, double *fx, double *fy, double *fz, double *vx, double *vy,
                 double *vz, int *err, hipStream_t st);
// f -= mean in place.
void launch_sub_mean(int64_t n, const double *mean, double *fx, double *fy, double *fz, hipStream_t st);
// v += h f; x <- wrap(x + dt v).
// Binning keys of the drifted positions, written by the drift kernels for the
// step's counting sort (key, run slot and histogram as the keys pass of
// launch_bin; the histogram must be cleared before). key == nullptr: none.
struct BinKeyOut {
  const double *q;
  int32_t *key, *slot, *count;
};
void launch_kick_kick_drift(int64_t n, double h, double dt, const Grid &g, const double *mean, const double *fx,
                            const double *fy, const double *fz, double *vx, double *vy, double *vz, double *x,
                            double *y, double *z, int *err, BinKeyOut bk, hipStream_t st);
// v <- s v + h f with s = *scale (nullptr: s = 1); x <- wrap(x + dt v).
void launch_kick_drift(int64_t n, double h, double dt, const Grid &g, const double *scale, const double *fx,
                       const double *fy, const double *fz, double *vx, double *vy, double *vz, double *x, double *y,
                       double *z, int *err, BinKeyOut bk, hipStream_t st);
// Nose-Hoover thermostat: constants of the half-steps.
struct NhParams {
  double dt, nf, kT, Q, mass;  // time step, degrees of freedom 3N - 3, target kT, thermostat mass, particle mass
};
enum { kNhStart = 1, kNhEnd = 2 };
int nh_part_len();
// Second half-kick (when h != 0; f -= mean written back when mean is given),
// K = (m/2) sum |v|^2, then the thermostat half-steps of `mode` on nh = {xi,
// eta} (device); *scale receives the velocity scaling still to apply.
void launch_nh(int64_t n, double h, const double *mean, double *fx, double *fy, double *fz, double *vx, double *vy,
               double *vz, const NhParams &q, int mode, double *part, double *nh, double *scale, int *err,
               hipStream_t st);
// v *= *scale.
void launch_scale_v(int64_t n, const double *scale, double *vx, double *vy, double *vz, hipStream_t st);
// Reorder the integrator state through perm (out[k] = in[perm[k]]).
struct StateArrays {
  double *x, *y, *z, *vx, *vy, *vz, *q;
  int32_t *id;
};

// ---------------------------------------------------------------------------
// batched form (many replicas, one persistent launch per step)
// ---------------------------------------------------------------------------
struct RepDesc {
  Grid g;
  int64_t p0, n;       // particle range
  int64_t c0;          // first key (2 * ncell keys per replica)
  Sten s_coul, s_lj;   // stencil radii
  ModeTable mt;        // mode table; its cdf starts at cdf_off
  int cdf_off;
  uint64_t seed;
  int nq;              // charged particles (the first nq of the replica's sorted range)
  int chunk_len;       // structure-factor chunk length
  int nchunks;         // chunks of this replica
  int chunk_off;       // first chunk of this replica in the partial array
  int rho_item_off;    // first structure-factor item of this replica
};

struct BatchArgs {
  int nrep;
  const RepDesc *reps;
  const int32_t *rep_of;  // replica of every particle slot
  int64_t ntot;
  int64_t nkeys;
  int ntiles;
  int P;
  int mode;               // 0: step, 1: force evaluation only
  int launch_part;        // launch of the step: 1 phases P0-P6, 2 phases P7-P9 (set by the launchers)
  const int *rho_items;   // total structure-factor items (chunk x 64-mode group), on the device
  int do_far;             // Fourier part on
  PairParams pp;          // physics shared by all replicas (grid fields unused)
  PairF32 pf;
  double h, dt;           // dt / (2 m), dt
  // state: in (read; advanced in place by the drift) and out (sorted)
  double *ix, *iy, *iz, *ivx, *ivy, *ivz, *iq, *ifx, *ify, *ifz;
  int32_t *iid;
  double *ox, *oy, *oz, *ovx, *ovy, *ovz, *oq, *ofx, *ofy, *ofz;
  int32_t *oid;
  double *cfx, *cfy, *cfz;  // force-only mode: output in the caller's order
  double4 *xq, *sq;
  int32_t *sid;
  int32_t *key, *slot, *tmp, *perm, *count, *cell_start, *tile_sum;
  const double *cdf;
  GatherMode *modes;      // [nrep * P]
  double *wk;             // [nrep * P] mode weights
  double2 *part;          // [total chunks * P]
  int *err;
  unsigned *bar;          // [2] arrival count, generation
  uint64_t *eval;         // evaluation index of the step (advanced by the kernel)
};

// Resident capacity of the step kernel (blocks), the launch, and the scan tiling.
int batch_grid_blocks(int prec, int device);
void launch_batch_step(int prec, int blocks, const BatchArgs &a, hipStream_t st);
int batch_scan_tiles(int64_t nkeys);
// Adds one step to `graph`: the first part of the step kernel, the near-field
// kernel and the second part, chained; *node is the last (the nodes copy *a).
hipError_t add_batch_node(hipGraph_t graph, hipGraphNode_t *node, const hipGraphNode_t *deps, int ndeps, int prec,
                          int blocks, BatchArgs *a);
// Per-replica charge statistics: nq[r] charged count, qs[2r] = sum q, qs[2r+1] = sum |q|.
void launch_qstats_rep(int nrep, const int64_t *off, const double *q, int32_t *nq, double *qs, hipStream_t st);
// Checks of Eq. 1 per replica (device error flags) and the structure-factor
// layout of every replica from the device counts (writes the nq, chunk and
// item fields of reps[] on the device, the item total and the first replica
// that failed a check, -1 if none).
void launch_batch_layout(int nrep, const int32_t *nq, const double *qs, int P, int chunk_len, RepDesc *reps,
                         int *rho_items, int *bad_rep, int *err, hipStream_t st);
// *p = v on the stream (a kernel, so graph capture records no memset node).
void launch_set_u64(uint64_t *p, uint64_t v, hipStream_t st);

// Error of a call without a context: the message rbe_last_error(NULL)
// returns, and the status code passed through.
int fail_without_context(int code, const char *msg);

}  // namespace rbe
