// C ABI of the RBE library: context management, validation and the
// orchestration of one force evaluation / one velocity-Verlet step.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

using namespace rbe;

namespace {

struct Buf {
  std::vector<void *> ptrs;
  bool ok = true;
  template <class T>
  T *alloc(int64_t count) {
    if (count <= 0) count = 1;
    void *p = nullptr;
    if (hipMalloc(&p, (size_t)count * sizeof(T)) != hipSuccess) {
      ok = false;
      return nullptr;
    }
    ptrs.push_back(p);
    return (T *)p;
  }
  void release() {
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

struct WorkSet {
  double *x, *y, *z, *vx, *vy, *vz, *q, *fx, *fy, *fz;
  int32_t *id;
  StateArrays arrays() const { return StateArrays{x, y, z, vx, vy, vz, q, id}; }
};

thread_local std::string g_create_error;

// Event pairs recorded around launches when timing is on; summed per kind.
struct Timer {
  bool on = false;
  std::vector<hipEvent_t> ev;
  std::vector<int> kind;  // kind of each recorded pair
  std::vector<int> count; // launches inside each recorded pair
  size_t used = 0;
  double ms[RBE_TIMING_KINDS] = {};
  int64_t launches[RBE_TIMING_KINDS] = {};
};

}  // namespace

struct rbe_ctx {
  int device = 0;
  rbe_params p{};
  int64_t n_max = 0;
  Grid g{};
  PairParams pp{};
  ModeTable mt{};
  std::vector<double> cdf_host;
  Buf buf;
  double *cdf_dev = nullptr;
  BinBuffers bb{};
  int32_t *cell_start = nullptr, *perm = nullptr, *inv_id = nullptr;
  Sorted srt{};
  WorkSet ws[2]{};
  FourierBuffers fb{};
  GhostBuffers gb{};
  bool ghosts = false;
  int32_t *m_dev = nullptr;  // [kSampleSteps][3][P] mode samples (rbe_step draws them ahead)
  double *w_dev = nullptr;   // [kSampleSteps][P]
  double *mkd_dev = nullptr; // [kSampleSteps][3][P] the same modes as doubles
  bool fixed_modes = false;  // rbe_set_modes: slot 0 of m_dev/w_dev/mkd_dev is the caller's table
  double *mean_part = nullptr, *mean = nullptr;
  double *epart = nullptr;   // energy partial sums
  double *nh_part = nullptr, *nh_scale = nullptr;  // thermostat: |v|^2 partials, pending velocity scaling
  int *err = nullptr;
  double *qstats = nullptr;  // [sum q, sum |q|]
  unsigned long long *counters = nullptr;
  bool counting = false;
  Timer tm;
  std::string last_error;
  // batched form (nrep > 1)
  struct Batch {
    int nrep = 0;
    std::vector<RepDesc> reps;  // host copy (the nq and chunk fields live on the device only)
    std::vector<int64_t> off;   // [nrep + 1]
    int64_t ntot = 0, nkeys = 0;
    int ntiles = 0, blocks = 0;
    int64_t part_chunks = 0;    // chunk capacity of the partial array
    RepDesc *reps_dev = nullptr;
    int32_t *rep_of = nullptr, *key = nullptr, *slot = nullptr, *tmp = nullptr, *count = nullptr;
    int32_t *tile_sum = nullptr, *nq = nullptr;
    int64_t *off_dev = nullptr;
    double *qs = nullptr, *wk = nullptr;
    GatherMode *modes = nullptr;
    double2 *part = nullptr;
    unsigned *bar = nullptr;
    uint64_t *eval = nullptr;
    int *rho_items = nullptr;  // device: structure-factor items of this call
    int *bad_rep = nullptr;    // device: first replica that failed the charge checks (-1: none)
    BatchArgs node_args[2]{};  // arguments of the two graph nodes
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
  } bt;
  bool batched() const { return bt.nrep > 0; }

  int fail(int code, const char *fmt, ...) __attribute__((format(printf, 3, 4)));
};

int rbe_ctx::fail(int code, const char *fmt, ...) {
  char msg[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(msg, sizeof msg, fmt, ap);
  va_end(ap);
  last_error = msg;
  return code;
}

static int create_fail(int code, const char *msg) {
  g_create_error = msg;
  return code;
}

int rbe::fail_without_context(int code, const char *msg) { return create_fail(code, msg); }

#define HIP_TRY(ctx, expr)                                                                     \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess)                                                                      \
      return (ctx)->fail(RBE_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));          \
  } while (0)

// ---------------------------------------------------------------------------
// per-kernel timing
// ---------------------------------------------------------------------------
static void timer_flush(rbe_ctx *c, hipStream_t st) {
  Timer &t = c->tm;
  if (t.used == 0) return;
  (void)hipStreamSynchronize(st);
  for (size_t k = 0; k < t.used / 2; ++k) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess) {
      t.ms[t.kind[k]] += ms;
      t.launches[t.kind[k]] += t.count[k];
    }
  }
  t.used = 0;
  t.kind.clear();
  t.count.clear();
}

// Evaluations whose mode samples rbe_step draws in one launch.
constexpr int kSampleSteps = 32;

struct TScope {
  rbe_ctx *c;
  hipStream_t st;
  bool on;
  TScope(rbe_ctx *c_, int kind, hipStream_t st_, int launches = 1) : c(c_), st(st_), on(c_->tm.on) {
    if (!on) return;
    Timer &t = c->tm;
    if (t.used + 2 > t.ev.size()) timer_flush(c, st);
    t.kind.push_back(kind);
    t.count.push_back(launches);
    (void)hipEventRecord(t.ev[t.used], st);
  }
  ~TScope() {
    if (!on) return;
    Timer &t = c->tm;
    (void)hipEventRecord(t.ev[t.used + 1], st);
    t.used += 2;
  }
};

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static int validate_params(const rbe_params *p, std::string *why) {
  char msg[256];
  auto bad = [&](int code, const char *m) {
    *why = m;
    return code;
  };
  for (int d = 0; d < 3; ++d)
    if (!(p->L[d] > 0) || !std::isfinite(p->L[d])) return bad(RBE_EINVAL, "box edges must be positive and finite");
  if (!(p->alpha > 0)) return bad(RBE_EINVAL, "alpha must be positive");
  if (!(p->r_coul > 0) || !(p->r_lj >= 0) || !(p->r_core >= 0)) return bad(RBE_EINVAL, "cutoffs must be positive");
  if (p->P < 1 || p->P > RBE_MAX_P) return bad(RBE_EINVAL, "P must be in [1, RBE_MAX_P]");
  if (p->kdist != RBE_KDIST_GAUSS && p->kdist != RBE_KDIST_GAUSS_OVER_K2)
    return bad(RBE_EINVAL, "kdist must be RBE_KDIST_GAUSS or RBE_KDIST_GAUSS_OVER_K2");
  if (p->prec != RBE_FP64 && p->prec != RBE_FP32C) return bad(RBE_EINVAL, "prec must be RBE_FP64 or RBE_FP32C");
  if (p->terms < 0 || p->terms > RBE_TERM_ALL) return bad(RBE_EINVAL, "bad term mask");
  if (p->rbl_shell != RBE_SHELL_ALL && p->rbl_shell != RBE_SHELL_CHARGED)
    return bad(RBE_EINVAL, "rbl_shell must be RBE_SHELL_ALL or RBE_SHELL_CHARGED");
  if (p->rbl_shell == RBE_SHELL_CHARGED && !(p->r_core > 0 && p->r_lj <= p->r_core))
    return bad(RBE_EINVAL, "a charged-only shell needs the random batch list and r_lj <= r_core");
  if (p->r_core > 0) {
    if (p->p_shell < 1 || p->p_shell > RBE_MAX_SHELL_BATCH) return bad(RBE_EINVAL, "p_shell must be in [1, 32]");
    if (p->r_core > p->r_coul) return bad(RBE_EINVAL, "r_core must not exceed r_coul");
    if (p->r_lj > p->r_coul) return bad(RBE_EINVAL, "with the random batch list r_lj must not exceed r_coul");
  }
  if (!(p->mass > 0) || !(p->dt >= 0)) return bad(RBE_EINVAL, "mass must be positive and dt non-negative");
  if (!(p->lj_sigma > 0) || !(p->lj_eps >= 0)) return bad(RBE_EINVAL, "bad LJ parameters");
  const double rmax = std::fmax(p->r_coul, p->r_lj);
  if (!(p->nvt_tau >= 0.0) || !std::isfinite(p->nvt_tau)) return bad(RBE_EINVAL, "nvt_tau must be >= 0 and finite");
  if (p->nvt_tau > 0.0 && (!(p->nvt_kT > 0.0) || !std::isfinite(p->nvt_kT)))
    return bad(RBE_EINVAL, "NVT needs a positive finite nvt_kT");
  if (!(p->ghost_width >= 0.0)) return bad(RBE_EINVAL, "ghost_width must be >= 0");
  if (p->ghost_width > 0.0) {
    if (p->ghost_width < rmax) return bad(RBE_EINVAL, "ghost_width must cover the largest cutoff");
    for (int d = 0; d < 3; ++d)
      if (p->ghost_width > 0.5 * p->L[d]) return bad(RBE_EBOX, "ghost_width exceeds half the box edge");
  }
  for (int d = 0; d < 3; ++d)
    if (rmax > 0.5 * p->L[d]) {
      snprintf(msg, sizeof msg, "cutoff %.6g exceeds half the box edge %.6g (minimum image)", rmax, p->L[d]);
      return bad(RBE_EBOX, msg);
    }
  for (int d = 0; d < 3; ++d)
    if (p->ncell[d] < 0) return bad(RBE_EINVAL, "ncell must be >= 0");
  if (std::sqrt(p->alpha) * p->r_coul > 8.0)
    return bad(RBE_EINVAL, "sqrt(alpha) r_coul must not exceed 8 (range of the erfc approximation)");
  return RBE_OK;
}

// Default grid: cell edge about max(r_lj, r_coul / 2) along y and z, and x
// cells kDefaultXSplit times finer (stencil rows are trimmed per particle
// along x, so finer x cells remove candidates without adding rows), as far
// as the cell table allows.
constexpr int kDefaultXSplit = 4;
static void choose_grid(const rbe_params *p, int nc[3]) {
  const bool user = p->ncell[0] > 0 && p->ncell[1] > 0 && p->ncell[2] > 0;
  const double h = std::fmax(p->r_lj, 0.5 * p->r_coul);
  for (int d = 0; d < 3; ++d) {
    if (user) {
      nc[d] = p->ncell[d];
    } else {
      int c = (int)std::floor(p->L[d] / h);
      nc[d] = c < 1 ? 1 : c;
    }
  }
  if (!user) {
    int k = kDefaultXSplit;
    while (k > 1 && (int64_t)k * nc[0] * nc[1] * nc[2] * 2 >= (1LL << 29)) --k;
    nc[0] *= k;
  }
}

static int stencil_radius(double r, double L, int n) {
  if (r <= 0) return 0;
  const double h = L / n;
  int s = (int)std::ceil(r / h * (1.0 + 1e-12));
  return s < 1 ? 1 : s;
}

// Pair constants and stencil radii of one grid (p->terms already defaulted).
static void make_pair_params(const rbe_params &p, const Grid &g, PairParams *out) {
  PairParams &pp = *out;
  pp = PairParams{};
  pp.g = g;
  const int nc[3] = {g.nx, g.ny, g.nz};
  const double rq = std::fmax(p.r_coul, p.r_lj);
  auto radii = [&](double r) {
    return Sten{stencil_radius(r, p.L[0], nc[0]), stencil_radius(r, p.L[1], nc[1]), stencil_radius(r, p.L[2], nc[2])};
  };
  pp.s_coul = radii(rq);
  pp.s_lj = radii(p.r_lj);
  pp.s_core = radii(std::fmax(p.r_core, p.r_lj));
  pp.rc2 = p.r_coul * p.r_coul;
  pp.rlj2 = p.r_lj * p.r_lj;
  pp.rcore2 = p.r_core * p.r_core;
  pp.rq2 = std::fmax(pp.rc2, pp.rlj2);
  pp.alpha = p.alpha;
  pp.sqrt_alpha = std::sqrt(p.alpha);
  pp.two_sqrt_alpha_over_sqrt_pi = 2.0 * pp.sqrt_alpha / std::sqrt(kPi);
  pp.kc = p.coulomb_k;
  pp.eps24 = 24.0 * p.lj_eps;
  pp.sig2 = p.lj_sigma * p.lj_sigma;
  pp.do_coul = (p.terms & RBE_TERM_COUL_REAL) != 0;
  pp.do_lj = (p.terms & RBE_TERM_LJ) != 0 && p.r_lj > 0;
  pp.rbl = p.r_core > 0;
  pp.shell_charged = pp.rbl && p.rbl_shell == RBE_SHELL_CHARGED;
  pp.p_shell = p.p_shell;
}

// Native cell grid of a box (no ghost layers).
static Grid make_grid(const rbe_params &p, const int nc[3]) {
  Grid g{};
  g.nx = nc[0];
  g.ny = nc[1];
  g.nz = nc[2];
  g.ncell = nc[0] * nc[1] * nc[2];
  for (int d = 0; d < 3; ++d) {
    g.L[d] = p.L[d];
    g.inv_h[d] = (double)nc[d] / p.L[d];
    g.goff[d] = 0;
  }
  g.pnx = g.nx;
  g.pny = g.ny;
  g.pnz = g.nz;
  g.pncell = g.ncell;
  g.ghost_width = 0.0;
  return g;
}

// Parameters, cell grid (with ghost layers when the shell is on) and pair
// constants of a single-system context (host only).
static int ctx_geometry(rbe_ctx *c, const rbe_params *p, int64_t n_max, std::string *why) {
  c->p = *p;
  if (c->p.terms == 0) c->p.terms = RBE_TERM_ALL;
  c->n_max = n_max;
  int nc[3];
  choose_grid(&c->p, nc);
  if ((int64_t)nc[0] * nc[1] * nc[2] >= (1LL << 29)) {
    *why = "cell grid too large";
    return RBE_EINVAL;
  }
  Grid &g = c->g;
  g.nx = nc[0];
  g.ny = nc[1];
  g.nz = nc[2];
  g.ncell = nc[0] * nc[1] * nc[2];
  for (int d = 0; d < 3; ++d) {
    g.L[d] = p->L[d];
    g.inv_h[d] = (double)nc[d] / p->L[d];
    c->p.ncell[d] = nc[d];
    // ghost layers: enough cells to hold every image within ghost_width
    g.goff[d] = p->ghost_width > 0 ? (int)std::ceil(p->ghost_width * g.inv_h[d] * (1.0 + 1e-12)) : 0;
  }
  g.ghost_width = p->ghost_width;
  make_pair_params(c->p, g, &c->pp);
  if (p->ghost_width > 0) {
    // the ghost layers must also hold every stencil
    const PairParams &q = c->pp;
    g.goff[0] = std::max(g.goff[0], std::max(q.s_coul.x, std::max(q.s_lj.x, q.s_core.x)));
    g.goff[1] = std::max(g.goff[1], std::max(q.s_coul.y, std::max(q.s_lj.y, q.s_core.y)));
    g.goff[2] = std::max(g.goff[2], std::max(q.s_coul.z, std::max(q.s_lj.z, q.s_core.z)));
  }
  g.pnx = g.nx + 2 * g.goff[0];
  g.pny = g.ny + 2 * g.goff[1];
  g.pnz = g.nz + 2 * g.goff[2];
  g.pncell = g.pnx * g.pny * g.pnz;
  if (p->ghost_width > 0 && (int64_t)g.pnx * g.pny * g.pnz >= (1LL << 29)) {
    *why = "padded cell grid too large";
    return RBE_EINVAL;
  }
  c->pp.g = g;
  return RBE_OK;
}

// ---------------------------------------------------------------------------
// create / destroy
// ---------------------------------------------------------------------------
extern "C" int rbe_create(rbe_ctx **out, const rbe_params *p, int64_t n_max, int device) {
  if (!out) return create_fail(RBE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!p) return create_fail(RBE_EINVAL, "params is NULL");
  if (n_max < 1 || n_max > (int64_t)0x7FFFFFFF) return create_fail(RBE_EINVAL, "n_max must be in [1, 2^31)");
  if (p && p->ghost_width > 0 && 8 * n_max >= (int64_t)0x7FFFFFFF)
    return create_fail(RBE_EINVAL, "with a ghost shell n_max must be below 2^28 (image offsets are 32-bit)");
  std::string why;
  int rc = validate_params(p, &why);
  if (rc != RBE_OK) return create_fail(rc, why.c_str());
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return create_fail(RBE_EDEVICE, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return create_fail(RBE_EDEVICE, "hipSetDevice failed");

  rbe_ctx *c = new rbe_ctx();
  c->device = device;
  rc = ctx_geometry(c, p, n_max, &why);
  if (rc != RBE_OK) {
    delete c;
    return create_fail(rc, why.c_str());
  }
  const Grid &g = c->g;

  // mode tables
  build_mode_table(p->L, p->alpha, &c->mt, nullptr);
  c->cdf_host.resize(c->mt.total);
  build_mode_table(p->L, p->alpha, &c->mt, c->cdf_host.data(), p->kdist);

  // device scratch
  Buf &b = c->buf;
  const int64_t nkeys = 2 * (int64_t)g.ncell;
  c->cdf_dev = b.alloc<double>(c->mt.total);
  c->bb.key = b.alloc<int32_t>(n_max);
  c->bb.slot = b.alloc<int32_t>(n_max);
  c->bb.tmp = b.alloc<int32_t>(n_max);
  c->bb.count = b.alloc<int32_t>(nkeys);
  c->bb.scan_tmp = b.alloc<int32_t>(scan_tiles(nkeys));
  c->cell_start = b.alloc<int32_t>(nkeys + 1);
  c->perm = b.alloc<int32_t>(n_max);
  c->inv_id = b.alloc<int32_t>(n_max);
  c->srt.xq = b.alloc<double4>(n_max + kScanPad);
  c->srt.sq = b.alloc<double4>(n_max);
  c->srt.id = b.alloc<int32_t>(n_max + kScanPad);
  for (int s = 0; s < 2; ++s) {
    WorkSet &w = c->ws[s];
    w.x = b.alloc<double>(n_max);
    w.y = b.alloc<double>(n_max);
    w.z = b.alloc<double>(n_max);
    w.vx = b.alloc<double>(n_max);
    w.vy = b.alloc<double>(n_max);
    w.vz = b.alloc<double>(n_max);
    w.q = b.alloc<double>(n_max);
    w.fx = b.alloc<double>(n_max);
    w.fy = b.alloc<double>(n_max);
    w.fz = b.alloc<double>(n_max);
    w.id = b.alloc<int32_t>(n_max);
  }
  const int P = p->P;
  int64_t nchunk = (n_max + 63) / 64;
  if (nchunk > 8192) nchunk = 8192;
  c->fb.nchunk_max = (int)nchunk;
  c->fb.mkd = b.alloc<double>(3 * P);
  // the partial launch never uses more chunks than this for any nq <= n_max
  c->fb.part = b.alloc<double2>((int64_t)rho_max_chunks(n_max, P, (int)nchunk) * P);
  c->fb.gpart = b.alloc<double4>(kGatherPartMax);
  c->fb.rho = b.alloc<double>(2 * P);
  c->fb.modes = b.alloc<GatherMode>(P);
  c->fb.turn_tab = b.alloc<double2>(kTurnTableEntries);
  c->m_dev = b.alloc<int32_t>((int64_t)kSampleSteps * 3 * P);
  c->w_dev = b.alloc<double>((int64_t)kSampleSteps * P);
  c->mkd_dev = b.alloc<double>((int64_t)kSampleSteps * 3 * P);
  c->mean_part = b.alloc<double>(3 * (int64_t)mean_blocks(n_max) + 3);
  c->mean = b.alloc<double>(3);
  c->epart = b.alloc<double>(energy_part_len(n_max));
  c->nh_part = b.alloc<double>(nh_part_len());
  c->nh_scale = b.alloc<double>(1);
  c->err = b.alloc<int>(1);
  c->qstats = b.alloc<double>(2);
  c->counters = b.alloc<unsigned long long>(12);
  if (p->ghost_width > 0) {
    // ghost capacity: the expected image count of a uniform fluid in the
    // shell (goff[d] cells thick) with 30 % headroom (at most 7 images per
    // native); overflow is flagged, and the cells past it are left empty
    double vol = 1.0;
    for (int d = 0; d < 3; ++d) vol *= 1.0 + 2.0 * g.goff[d] * (p->L[d] / (d == 0 ? g.nx : d == 1 ? g.ny : g.nz)) / p->L[d];
    int64_t cap = (int64_t)std::ceil(1.3 * (double)n_max * (vol - 1.0)) + 4096;
    if (cap > 7 * n_max + 4096) cap = 7 * n_max + 4096;
    if (cap + n_max >= (int64_t)0x7FFFFFFF) cap = (int64_t)0x7FFFFFFF - n_max - 1;
    GhostBuffers &gb = c->gb;
    gb.cap = cap;
    const int64_t pkeys = 2 * (int64_t)g.pncell;
    gb.xq = b.alloc<double4>(cap + kScanPad);
    gb.id = b.alloc<int32_t>(cap + kScanPad);
    gb.cell_start = b.alloc<int32_t>(pkeys + 1);
    gb.cell_count = b.alloc<int32_t>(pkeys);
    gb.cell_scan_tmp = b.alloc<int32_t>(scan_tiles(pkeys));
    gb.count = b.alloc<int32_t>(1);
    c->ghosts = true;
  }
  if (!b.ok) {
    b.release();
    delete c;
    return create_fail(RBE_ENOMEM, "device allocation failed");
  }
  double2 turn_host[kTurnTableEntries];
  fill_turn_table(turn_host, kTurnTableEntries);
  if (hipMemcpy(c->cdf_dev, c->cdf_host.data(), sizeof(double) * c->mt.total, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(c->fb.turn_tab, turn_host, sizeof turn_host, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(c->err, 0, sizeof(int)) != hipSuccess ||
      hipMemset(c->counters, 0, 12 * sizeof(unsigned long long)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    b.release();
    delete c;
    return create_fail(RBE_EDEVICE, "initial device copies failed");
  }
  *out = c;
  return RBE_OK;
}

// Structure-factor chunk length of the batched form (particles per wave item).
constexpr int kBatchChunk = 128;

static bool same_shared_physics(const rbe_params &a, const rbe_params &b) {
  auto t = [](int v) { return v == 0 ? RBE_TERM_ALL : v; };
  return a.alpha == b.alpha && a.r_coul == b.r_coul && a.r_lj == b.r_lj && a.r_core == b.r_core &&
         a.p_shell == b.p_shell && a.P == b.P && a.kdist == b.kdist && a.prec == b.prec && t(a.terms) == t(b.terms) &&
         a.lj_eps == b.lj_eps && a.lj_sigma == b.lj_sigma && a.coulomb_k == b.coulomb_k && a.mass == b.mass &&
         a.dt == b.dt && a.ghost_width == b.ghost_width && a.nvt_kT == b.nvt_kT && a.nvt_tau == b.nvt_tau;
}

extern "C" int rbe_create_batch(rbe_ctx **out, int32_t n_sys, const rbe_params *params, const int64_t *offset,
                                int device) {
  if (!out) return create_fail(RBE_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params || !offset) return create_fail(RBE_EINVAL, "params or offset is NULL");
  if (n_sys < 1) return create_fail(RBE_EINVAL, "n_sys must be >= 1");
  if (offset[0] != 0) return create_fail(RBE_EINVAL, "offset[0] must be 0");
  for (int32_t r = 0; r < n_sys; ++r)
    if (offset[r + 1] <= offset[r]) return create_fail(RBE_EINVAL, "every replica needs at least one particle");
  if (offset[n_sys] >= (int64_t)0x7FFFFFFF) return create_fail(RBE_EINVAL, "total particle count must be < 2^31");
  if (n_sys == 1) return rbe_create(out, params, offset[1], device);
  std::string why;
  char msg[400];
  for (int32_t r = 0; r < n_sys; ++r) {
    const int rc = validate_params(&params[r], &why);
    if (rc != RBE_OK) {
      snprintf(msg, sizeof msg, "replica %d: %s", (int)r, why.c_str());
      return create_fail(rc, msg);
    }
    if (!same_shared_physics(params[r], params[0])) {
      snprintf(msg, sizeof msg, "replica %d differs from replica 0 in a field other than L, ncell and seed", (int)r);
      return create_fail(RBE_EINVAL, msg);
    }
  }
  if (params[0].r_core > 0)
    return create_fail(RBE_EINVAL, "the random batch list (r_core > 0) is not available in the batched form");
  if (params[0].ghost_width > 0)
    return create_fail(RBE_EINVAL, "the ghost shell (ghost_width > 0) is not available in the batched form");
  if (params[0].nvt_tau > 0)
    return create_fail(RBE_EINVAL, "the NVT thermostat (nvt_tau > 0) is not available in the batched form");
  if (params[0].kdist != RBE_KDIST_GAUSS)
    return create_fail(RBE_EINVAL, "the batched form samples the Gaussian mode distribution only");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return create_fail(RBE_EDEVICE, "no such HIP device");
  if (hipSetDevice(device) != hipSuccess) return create_fail(RBE_EDEVICE, "hipSetDevice failed");

  rbe_ctx *c = new rbe_ctx();
  c->device = device;
  c->p = params[0];
  if (c->p.terms == 0) c->p.terms = RBE_TERM_ALL;
  auto &B = c->bt;
  B.nrep = n_sys;
  B.off.assign(offset, offset + n_sys + 1);
  B.ntot = offset[n_sys];
  c->n_max = B.ntot;
  std::vector<double> cdf_all;
  int64_t key0 = 0, chunks = 0;
  B.reps.resize(n_sys);
  for (int32_t r = 0; r < n_sys; ++r) {
    rbe_params pr = params[r];
    pr.terms = c->p.terms;
    int nc[3];
    choose_grid(&pr, nc);
    if ((int64_t)nc[0] * nc[1] * nc[2] >= (1LL << 29)) {
      delete c;
      return create_fail(RBE_EINVAL, "cell grid too large");
    }
    RepDesc &d = B.reps[r];
    d = RepDesc{};
    d.g = make_grid(pr, nc);
    PairParams pr_pp;
    make_pair_params(pr, d.g, &pr_pp);
    d.s_coul = pr_pp.s_coul;
    d.s_lj = pr_pp.s_lj;
    d.p0 = offset[r];
    d.n = offset[r + 1] - offset[r];
    d.c0 = key0;
    key0 += 2 * (int64_t)d.g.ncell;
    build_mode_table(pr.L, pr.alpha, &d.mt, nullptr);
    d.cdf_off = (int)cdf_all.size();
    cdf_all.resize(cdf_all.size() + d.mt.total);
    build_mode_table(pr.L, pr.alpha, &d.mt, cdf_all.data() + d.cdf_off);
    d.seed = pr.seed;
    chunks += (d.n + kBatchChunk - 1) / kBatchChunk;
    if (r == 0) {
      c->g = d.g;
      c->pp = pr_pp;
      c->mt = d.mt;
    }
  }
  if (key0 >= (int64_t)0x7FFFFFFF - 1) {
    delete c;
    return create_fail(RBE_EINVAL, "cell grids too large");
  }
  B.nkeys = key0;
  B.ntiles = batch_scan_tiles(key0);
  B.part_chunks = chunks;
  const int64_t n = B.ntot;
  const int P = c->p.P;

  Buf &b = c->buf;
  for (int s = 0; s < 2; ++s) {
    WorkSet &w = c->ws[s];
    w.x = b.alloc<double>(n);
    w.y = b.alloc<double>(n);
    w.z = b.alloc<double>(n);
    w.vx = b.alloc<double>(n);
    w.vy = b.alloc<double>(n);
    w.vz = b.alloc<double>(n);
    w.q = b.alloc<double>(n);
    w.fx = b.alloc<double>(n);
    w.fy = b.alloc<double>(n);
    w.fz = b.alloc<double>(n);
    w.id = b.alloc<int32_t>(n);
  }
  c->srt.xq = b.alloc<double4>(n + kScanPad);
  c->srt.sq = b.alloc<double4>(n);
  c->srt.id = b.alloc<int32_t>(n + kScanPad);
  c->perm = b.alloc<int32_t>(n);
  c->cell_start = b.alloc<int32_t>(B.nkeys + 1);
  c->cdf_dev = b.alloc<double>((int64_t)cdf_all.size());
  c->err = b.alloc<int>(1);
  c->counters = b.alloc<unsigned long long>(12);
  B.key = b.alloc<int32_t>(n);
  B.slot = b.alloc<int32_t>(n);
  B.tmp = b.alloc<int32_t>(n);
  B.count = b.alloc<int32_t>(B.nkeys);
  B.tile_sum = b.alloc<int32_t>(B.ntiles);
  B.rep_of = b.alloc<int32_t>(n);
  B.reps_dev = b.alloc<RepDesc>(n_sys);
  B.off_dev = b.alloc<int64_t>(n_sys + 1);
  B.nq = b.alloc<int32_t>(n_sys);
  B.qs = b.alloc<double>(2 * (int64_t)n_sys);
  B.modes = b.alloc<GatherMode>((int64_t)n_sys * P);
  B.wk = b.alloc<double>((int64_t)n_sys * P);
  B.part = b.alloc<double2>(chunks * P);
  B.bar = b.alloc<unsigned>(2);
  B.eval = b.alloc<uint64_t>(1);
  B.rho_items = b.alloc<int>(1);
  B.bad_rep = b.alloc<int>(1);
  if (!b.ok) {
    b.release();
    delete c;
    return create_fail(RBE_ENOMEM, "device allocation failed");
  }
  std::vector<int32_t> rep_of(n);
  for (int32_t r = 0; r < n_sys; ++r)
    for (int64_t i = offset[r]; i < offset[r + 1]; ++i) rep_of[i] = r;
  B.blocks = batch_grid_blocks(c->p.prec, device);
  if (hipMemcpy(c->cdf_dev, cdf_all.data(), sizeof(double) * cdf_all.size(), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B.rep_of, rep_of.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B.off_dev, offset, sizeof(int64_t) * (n_sys + 1), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(B.reps_dev, B.reps.data(), sizeof(RepDesc) * n_sys, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemset(B.count, 0, sizeof(int32_t) * B.nkeys) != hipSuccess ||
      hipMemset(B.bar, 0, 2 * sizeof(unsigned)) != hipSuccess || hipMemset(c->err, 0, sizeof(int)) != hipSuccess ||
      hipMemset(c->counters, 0, 12 * sizeof(unsigned long long)) != hipSuccess ||
      hipDeviceSynchronize() != hipSuccess) {
    b.release();
    delete c;
    return create_fail(RBE_EDEVICE, "initial device copies failed");
  }
  *out = c;
  return RBE_OK;
}

extern "C" void rbe_destroy(rbe_ctx *ctx) {
  if (!ctx) return;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->bt.exec) (void)hipGraphExecDestroy(ctx->bt.exec);
  if (ctx->bt.graph) (void)hipGraphDestroy(ctx->bt.graph);
  ctx->buf.release();
  for (auto &e : ctx->tm.ev) (void)hipEventDestroy(e);
  delete ctx;
}

extern "C" const char *rbe_last_error(const rbe_ctx *ctx) {
  if (!ctx) return g_create_error.c_str();
  return ctx->last_error.c_str();
}

// ---------------------------------------------------------------------------
// charge checks (on the device: no call waits for them)
// ---------------------------------------------------------------------------
// stats[0] += sum q, stats[1] += sum |q| (one atomic per wave, in any order:
// the sums only feed the neutrality test below); a non-finite charge raises
// kErrNonFinite.
__global__ void __launch_bounds__(256) k_qstats(int64_t n, const double *__restrict__ q, double *stats, int *err) {
  double s = 0.0, a = 0.0;
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double v = q[i];
    bad |= !isfinite(v);
    s += v;
    a += fabs(v);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    s += __shfl_xor(s, o, 64);
    a += __shfl_xor(a, o, 64);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) atomicOr(err, kErrNonFinite);
  if ((threadIdx.x & 63) == 0) {
    atomicAdd(&stats[0], s);
    atomicAdd(&stats[1], a);
  }
}

// Eq. 1 asks for a neutral system: |sum q| above 1e-10 sum |q| (and above
// 1e-12) raises kErrNonNeutral.
__global__ void k_qstatus(const double *__restrict__ stats, int *err) {
  const double s = stats[0], a = stats[1];
  if (isfinite(s) && isfinite(a) && fabs(s) > 1e-10 * fmax(a, 1e-300) && fabs(s) > 1e-12)
    atomicOr(err, kErrNonNeutral);
}

// Neutrality and finiteness of the charges, reported through the device flag
// that rbe_sync_check reads (the counts that size the later launches are read
// on the device too, so nothing here waits).
static void launch_charge_check(rbe_ctx *c, int64_t n, const double *q, hipStream_t st) {
  launch_fill_f64(c->qstats, 2, 0.0, st);
  int64_t blocks = (n + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  if (blocks < 1) blocks = 1;
  k_qstats<<<(unsigned)blocks, 256, 0, st>>>(n, q, c->qstats, c->err);
  k_qstatus<<<1, 1, 0, st>>>(c->qstats, c->err);
}

// ---------------------------------------------------------------------------
// one force evaluation on sorted data (ws[1] receives the sorted force)
// ---------------------------------------------------------------------------
// Inputs in c->srt (xq, sq, id) and c->cell_start; output in fx/fy/fz (sorted).
// inv_ready: the id -> slot map was already written (by the step's reorder)
// and the ids were validated earlier in the same call. mkd_pre: the modes m
// as doubles, drawn ahead by rbe_step (then m and w are that draw).
static int eval_sorted(rbe_ctx *c, int64_t n, const int32_t *m, const double *w, uint64_t eval,
                       double *rho_out, double *fx, double *fy, double *fz, hipStream_t st, bool inv_ready = false,
                       const double *mkd_pre = nullptr) {
  const int P = c->p.P;
  const int terms = c->p.terms;
  // charged particles come first in the cell order: their count is the
  // start of the first neutral cell
  const int32_t *nq = c->cell_start + c->g.ncell;
  if (terms & (RBE_TERM_LJ | RBE_TERM_COUL_REAL)) {
    PairParams pp = c->pp;
    pp.shell_key = shell_eval_key(c->p.seed, eval);
    // the mean shell holds particles of the shell's population: all (the
    // charged-only variant derives its threshold from the device count)
    pp.shell_T0 = shell_first_threshold(pp, n);
    if (pp.rbl && !inv_ready) {
      TScope ts(c, RBE_TK_REORDER, st);
      launch_inverse_ids(n, c->srt.id, c->inv_id, c->err, st);
    }
    const GhostBuffers *gb = nullptr;
    if (c->ghosts) {
      TScope ts(c, RBE_TK_GHOST, st);
      launch_build_ghosts(c->g, n, c->cell_start, c->srt, c->gb, c->err, st);
      gb = &c->gb;
    }
    if (c->counting) launch_fill_i32((int32_t *)c->counters, 24, 0, st);
    auto part_cnt = [&](int part) { return PairCounters{c->counting ? c->counters + 4 * part : nullptr}; };
    const bool tiles = lj_tile_applicable(c->p.prec, pp, n);
    if (!pp.rbl && tiles) {
      // LJ terms of every particle over LDS-staged cell tiles, then the
      // screened Coulomb terms of the charged particles added
      {
        TScope ts(c, RBE_TK_PAIR, st);
        launch_lj_tile(pp, n, 3, c->srt, c->cell_start, gb, fx, fy, fz, part_cnt(PAIR_PART_NEUTRAL).c,
                       c->err, st);
      }
      if (pp.do_coul) {
        TScope ts(c, RBE_TK_PAIR_CHARGED, st);
        launch_pair(c->p.prec, PAIR_PART_COULOMB, pp, n, nq, c->srt, c->cell_start, c->inv_id, gb, fx, fy, fz,
                    part_cnt(PAIR_PART_CHARGED), st);
      }
    } else {
      {
        TScope ts(c, RBE_TK_PAIR_CHARGED, st);
        launch_pair(c->p.prec, PAIR_PART_CHARGED, pp, n, nq, c->srt, c->cell_start, c->inv_id, gb, fx, fy, fz,
                    part_cnt(PAIR_PART_CHARGED), st);
      }
      {
        // neutral particles: LJ over the tiles when all their LJ terms lie in
        // the core (list on) or always (list off), else the list's cluster walk
        TScope ts(c, RBE_TK_PAIR, st);
        if (tiles && pp.rbl && !(pp.rlj2 > pp.rcore2))
          launch_lj_tile(pp, n, 2, c->srt, c->cell_start, gb, fx, fy, fz,
                         part_cnt(PAIR_PART_NEUTRAL).c, c->err, st);
        else
          launch_pair(c->p.prec, PAIR_PART_NEUTRAL, pp, n, nq, c->srt, c->cell_start, c->inv_id, gb, fx, fy, fz,
                      part_cnt(PAIR_PART_NEUTRAL), st);
      }
    }
    if (pp.rbl) {
      TScope ts(c, RBE_TK_MEAN, st);
      launch_mean3(n, fx, fy, fz, c->mean_part, c->mean, st);
    }
  } else {
    launch_fill_f64(fx, n, 0.0, st);
    launch_fill_f64(fy, n, 0.0, st);
    launch_fill_f64(fz, n, 0.0, st);
  }
  if (terms & RBE_TERM_FOURIER) {
    FourierBuffers fb = c->fb;
    if (mkd_pre) {
      fb.mkd = const_cast<double *>(mkd_pre);  // drawn ahead with the modes
    } else if (!m && c->fixed_modes) {
      m = c->m_dev;  // the fixed table (rbe_set_modes), converted when it was set
      w = c->w_dev;
      fb.mkd = c->mkd_dev;
    } else {
      TScope ts(c, RBE_TK_SAMPLE, st);
      if (!m) {
        launch_sample_modes(c->mt, c->cdf_dev, c->p.seed, eval, P, c->m_dev, c->w_dev, c->err, st);
        m = c->m_dev;
        w = c->w_dev;
      }
      launch_modes_to_double(P, m, fb.mkd, st);
    }
    {
      TScope ts(c, RBE_TK_RHO_PARTIAL, st);
      launch_rho_partial(c->p.prec, nq, n, P, c->srt.sq, fb, st);
    }
    {
      TScope ts(c, RBE_TK_RHO_FINAL, st);
      launch_rho_final(nq, P, fb, w, c->p.coulomb_k, rho_out, st);
    }
    {
      TScope ts(c, RBE_TK_GATHER, st);
      launch_fourier_gather(c->p.prec, nq, n, P, c->srt.sq, fb, c->g, fx, fy, fz, st);
    }
  }
  return RBE_OK;
}

static bool state_ok(const rbe_state *s, bool need_v) {
  if (!s || !s->x || !s->y || !s->z || !s->fx || !s->fy || !s->fz || !s->q || !s->id) return false;
  if (need_v && (!s->vx || !s->vy || !s->vz)) return false;
  return true;
}

extern "C" int rbe_build_cells(rbe_ctx *c, const double *x, const double *y, const double *z, const double *q,
                               int64_t n, int32_t *cell_start, int32_t *perm, void *stream) {
  if (!c) return RBE_EINVAL;
  if (n < 0 || n > c->n_max) return c->fail(RBE_ERANGE, "n = %lld outside [0, n_max = %lld]", (long long)n,
                                            (long long)c->n_max);
  if (n > 0 && (!x || !y || !z || !q || !perm)) return c->fail(RBE_EINVAL, "null array");
  if (!cell_start) return c->fail(RBE_EINVAL, "null cell_start");
  if (c->batched()) return c->fail(RBE_EINVAL, "rbe_build_cells is not available on a batched context");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  launch_bin(c->bb, c->g, n, x, y, z, q, cell_start, perm, st);
  HIP_TRY(c, hipGetLastError());
  return RBE_OK;
}

extern "C" int rbe_sample_k(const rbe_params *p, uint64_t eval, int32_t *m, double *w, int on_device, void *stream) {
  if (!p || !m || !w) return create_fail(RBE_EINVAL, "null argument");
  if (p->P < 1 || p->P > RBE_MAX_P || !(p->alpha > 0)) return create_fail(RBE_EINVAL, "bad P or alpha");
  for (int d = 0; d < 3; ++d)
    if (!(p->L[d] > 0)) return create_fail(RBE_EINVAL, "bad box");
  if (p->kdist != RBE_KDIST_GAUSS && p->kdist != RBE_KDIST_GAUSS_OVER_K2)
    return create_fail(RBE_EINVAL, "kdist must be RBE_KDIST_GAUSS or RBE_KDIST_GAUSS_OVER_K2");
  ModeTable t{};
  build_mode_table(p->L, p->alpha, &t, nullptr);
  std::vector<double> cdf(t.total);
  build_mode_table(p->L, p->alpha, &t, cdf.data(), p->kdist);
  if (!on_device) {
    if (sample_modes_host(t, cdf.data(), p->seed, eval, p->P, m, w) != 0)
      return create_fail(RBE_EINVAL, "mode sampler rejected every attempt");
    return RBE_OK;
  }
  hipStream_t st = (hipStream_t)stream;
  double *cdf_dev = nullptr;
  int *err = nullptr;
  if (hipMalloc(&cdf_dev, sizeof(double) * t.total) != hipSuccess) return create_fail(RBE_ENOMEM, "hipMalloc");
  if (hipMalloc(&err, sizeof(int)) != hipSuccess) {
    (void)hipFree(cdf_dev);
    return create_fail(RBE_ENOMEM, "hipMalloc");
  }
  int rc = RBE_OK;
  int herr = 0;
  if (hipMemcpyAsync(cdf_dev, cdf.data(), sizeof(double) * t.total, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(err, 0, sizeof(int), st) != hipSuccess)
    rc = create_fail(RBE_EDEVICE, "copy of the mode table failed");
  if (rc == RBE_OK) {
    launch_sample_modes(t, cdf_dev, p->seed, eval, p->P, m, w, err, st);
    if (hipMemcpyAsync(&herr, err, sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = create_fail(RBE_EDEVICE, "device sampler failed");
    else if (herr)
      rc = create_fail(RBE_EINVAL, "mode sampler rejected every attempt");
  }
  (void)hipFree(cdf_dev);
  (void)hipFree(err);
  return rc;
}

// ---------------------------------------------------------------------------
// batched form
// ---------------------------------------------------------------------------
// Per-replica charge statistics, the checks of Eq. 1 (device error flags) and
// the structure-factor chunk layout of this call, all on the device.
static void batch_prepare(rbe_ctx *c, const double *q, hipStream_t st) {
  auto &B = c->bt;
  launch_qstats_rep(B.nrep, B.off_dev, q, B.nq, B.qs, st);
  launch_batch_layout(B.nrep, B.nq, B.qs, c->p.P, kBatchChunk, B.reps_dev, B.rho_items, B.bad_rep, c->err, st);
}

// Launch arguments shared by both modes; the caller sets the state arrays.
static BatchArgs batch_args(rbe_ctx *c, int mode) {
  auto &B = c->bt;
  BatchArgs a{};
  a.nrep = B.nrep;
  a.reps = B.reps_dev;
  a.rep_of = B.rep_of;
  a.ntot = B.ntot;
  a.nkeys = B.nkeys;
  a.ntiles = B.ntiles;
  a.P = c->p.P;
  a.mode = mode;
  a.rho_items = B.rho_items;
  a.do_far = (c->p.terms & RBE_TERM_FOURIER) != 0;
  a.pp = c->pp;
  a.pf = make_pair_f32(a.pp);
  a.h = 0.5 * c->p.dt / c->p.mass;
  a.dt = c->p.dt;
  a.xq = c->srt.xq;
  a.sq = c->srt.sq;
  a.sid = c->srt.id;
  a.key = B.key;
  a.slot = B.slot;
  a.tmp = B.tmp;
  a.perm = c->perm;
  a.count = B.count;
  a.cell_start = c->cell_start;
  a.tile_sum = B.tile_sum;
  a.cdf = c->cdf_dev;
  a.modes = B.modes;
  a.wk = B.wk;
  a.part = B.part;
  a.err = c->err;
  a.bar = B.bar;
  a.eval = B.eval;
  return a;
}

static BatchArgs batch_step_args(rbe_ctx *c, const WorkSet &in, const WorkSet &out) {
  BatchArgs a = batch_args(c, 0);
  a.ix = in.x;
  a.iy = in.y;
  a.iz = in.z;
  a.ivx = in.vx;
  a.ivy = in.vy;
  a.ivz = in.vz;
  a.iq = in.q;
  a.ifx = in.fx;
  a.ify = in.fy;
  a.ifz = in.fz;
  a.iid = in.id;
  a.ox = out.x;
  a.oy = out.y;
  a.oz = out.z;
  a.ovx = out.vx;
  a.ovy = out.vy;
  a.ovz = out.vz;
  a.oq = out.q;
  a.ofx = out.fx;
  a.ofy = out.fy;
  a.ofz = out.fz;
  a.oid = out.id;
  return a;
}

// Start of a batched call: eval, barrier and histogram start from known values.
static int batch_begin(rbe_ctx *c, uint64_t eval, hipStream_t st) {
  auto &B = c->bt;
  launch_set_u64(B.eval, eval, st);
  launch_fill_i32((int32_t *)B.bar, 2, 0, st);
  launch_fill_i32(B.count, B.nkeys, 0, st);
  return RBE_OK;
}

// Two-step graph (ws[0] -> ws[1] -> ws[0]), instantiated on the first call
// with two or more steps (the layout it depends on is read on the device).
static int batch_graph(rbe_ctx *c) {
  auto &B = c->bt;
  if (B.exec) return RBE_OK;
  B.node_args[0] = batch_step_args(c, c->ws[0], c->ws[1]);
  B.node_args[1] = batch_step_args(c, c->ws[1], c->ws[0]);
  HIP_TRY(c, hipGraphCreate(&B.graph, 0));
  hipGraphNode_t n0 = nullptr, n1 = nullptr;
  HIP_TRY(c, add_batch_node(B.graph, &n0, nullptr, 0, c->p.prec, B.blocks, &B.node_args[0]));
  HIP_TRY(c, add_batch_node(B.graph, &n1, &n0, 1, c->p.prec, B.blocks, &B.node_args[1]));
  HIP_TRY(c, hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
  return RBE_OK;
}

static int batch_forces(rbe_ctx *c, const rbe_state *s, const int32_t *m, const double *w, uint64_t eval,
                        double *rho_out, hipStream_t st) {
  auto &B = c->bt;
  if (m || w || rho_out) return c->fail(RBE_EINVAL, "a batched context draws its own modes: m, w, rho_out must be NULL");
  if (s->n != B.ntot) return c->fail(RBE_ERANGE, "n = %lld, the batch holds %lld", (long long)s->n, (long long)B.ntot);
  batch_prepare(c, s->q, st);
  const int rc = batch_begin(c, eval, st);
  if (rc != RBE_OK) return rc;
  BatchArgs a = batch_args(c, 1);
  a.ix = s->x;
  a.iy = s->y;
  a.iz = s->z;
  a.iq = s->q;
  a.iid = s->id;
  const WorkSet &o = c->ws[1];
  a.ox = o.x;
  a.oy = o.y;
  a.oz = o.z;
  a.oq = o.q;
  a.oid = o.id;
  a.ofx = o.fx;
  a.ofy = o.fy;
  a.ofz = o.fz;
  a.cfx = s->fx;
  a.cfy = s->fy;
  a.cfz = s->fz;
  {
    TScope ts(c, RBE_TK_BATCH, st);
    launch_batch_step(c->p.prec, B.blocks, a, st);
  }
  HIP_TRY(c, hipGetLastError());
  return RBE_OK;
}

static int copy_state(rbe_ctx *c, const double *const src[10], const int32_t *sid, double *const dst[10],
                      int32_t *did, int64_t n, hipStream_t st) {
  for (int k = 0; k < 10; ++k)
    HIP_TRY(c, hipMemcpyAsync(dst[k], src[k], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(did, sid, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
  return RBE_OK;
}

// Batched steps without copying the state: the first step reads the caller's
// arrays and reorders into ws[0], the steps between alternate between the
// working sets (pairs of them through the two-step graph), and the last step
// reorders into the caller's arrays. A single step copies the state into
// ws[0] first.
static int batch_step(rbe_ctx *c, rbe_state *s, int32_t nsteps, uint64_t first_eval, hipStream_t st) {
  auto &B = c->bt;
  if (s->n != B.ntot) return c->fail(RBE_ERANGE, "n = %lld, the batch holds %lld", (long long)s->n, (long long)B.ntot);
  batch_prepare(c, s->q, st);
  const int64_t n = s->n;
  WorkSet S{s->x, s->y, s->z, s->vx, s->vy, s->vz, s->q, s->fx, s->fy, s->fz, s->id};
  int rc = batch_begin(c, first_eval, st);
  if (rc != RBE_OK) return rc;
  auto direct = [&](const WorkSet &in, const WorkSet &out) {
    BatchArgs a = batch_step_args(c, in, out);
    TScope ts(c, RBE_TK_BATCH, st);
    launch_batch_step(c->p.prec, B.blocks, a, st);
  };
  if (nsteps == 1) {
    WorkSet &A = c->ws[0];
    const double *src[10] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->fx, s->fy, s->fz, s->q};
    double *dst[10] = {A.x, A.y, A.z, A.vx, A.vy, A.vz, A.fx, A.fy, A.fz, A.q};
    rc = copy_state(c, src, s->id, dst, A.id, n, st);
    if (rc != RBE_OK) return rc;
    direct(A, S);
  } else {
    direct(S, c->ws[0]);
    const int32_t middle = nsteps - 2;
    if (middle >= 2) {
      rc = batch_graph(c);
      if (rc != RBE_OK) return rc;
      for (int32_t k = 0; k + 1 < middle; k += 2) {
        TScope ts(c, RBE_TK_BATCH, st, 2);
        HIP_TRY(c, hipGraphLaunch(B.exec, st));
      }
    }
    const WorkSet *cur = &c->ws[0];
    if (middle & 1) {
      direct(c->ws[0], c->ws[1]);
      cur = &c->ws[1];
    }
    direct(*cur, S);
  }
  HIP_TRY(c, hipGetLastError());
  return RBE_OK;
}

extern "C" int rbe_lattice_modes(const rbe_params *p, double k_max, int32_t *m, double *w, int32_t cap,
                                 int32_t *count) {
  if (!p || !count) return create_fail(RBE_EINVAL, "null argument");
  if (!(p->alpha > 0) || !(k_max > 0) || !std::isfinite(k_max)) return create_fail(RBE_EINVAL, "bad alpha or k_max");
  for (int d = 0; d < 3; ++d)
    if (!(p->L[d] > 0) || !std::isfinite(p->L[d])) return create_fail(RBE_EINVAL, "bad box");
  const double two_pi = 6.283185307179586476925286766559005768;
  int64_t M[3];
  for (int d = 0; d < 3; ++d) {
    const double md = std::floor(k_max * p->L[d] / two_pi);
    if (md > 4096) return create_fail(RBE_ERANGE, "k_max spans more than 4096 modes along an axis");
    M[d] = (int64_t)md;
  }
  const double V = p->L[0] * p->L[1] * p->L[2];
  const double k2max = k_max * k_max;
  int64_t cnt = 0;
  // half space: m_x > 0, or m_x = 0 and m_y > 0, or m_x = m_y = 0 and m_z > 0;
  // each mode stands for itself and its negative (same term), so its weight
  // is twice the Ewald coefficient
  for (int64_t mx = 0; mx <= M[0]; ++mx)
    for (int64_t my = mx ? -M[1] : 0; my <= M[1]; ++my)
      for (int64_t mz = (mx || my) ? -M[2] : 1; mz <= M[2]; ++mz) {
        const double kx = two_pi * (double)mx / p->L[0], ky = two_pi * (double)my / p->L[1],
                     kz = two_pi * (double)mz / p->L[2];
        const double k2 = kx * kx + ky * ky + kz * kz;
        if (k2 > k2max) continue;
        if (m) {
          if (cnt >= cap) return create_fail(RBE_ERANGE, "cap is smaller than the mode count");
          m[cnt] = (int32_t)mx;
          m[cap + cnt] = (int32_t)my;
          m[2 * (int64_t)cap + cnt] = (int32_t)mz;
          w[cnt] = 2.0 * 4.0 * M_PI * std::exp(-k2 / (4.0 * p->alpha)) / (V * k2);
        }
        ++cnt;
      }
  if (cnt > INT32_MAX) return create_fail(RBE_ERANGE, "mode count exceeds int32");
  *count = (int32_t)cnt;
  if (m && cnt != cap) return create_fail(RBE_ERANGE, "cap must equal the mode count");
  return RBE_OK;
}

extern "C" int rbe_set_modes(rbe_ctx *c, const int32_t *m, const double *w, void *stream) {
  if (!c) return RBE_EINVAL;
  if (c->batched()) return c->fail(RBE_EINVAL, "rbe_set_modes is not available on a batched context");
  if ((m == nullptr) != (w == nullptr)) return c->fail(RBE_EINVAL, "m and w must both be given or both be NULL");
  if (!m) {
    c->fixed_modes = false;
    return RBE_OK;
  }
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t P = c->p.P;
  HIP_TRY(c, hipMemcpyAsync(c->m_dev, m, sizeof(int32_t) * 3 * P, hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(c->w_dev, w, sizeof(double) * P, hipMemcpyDeviceToDevice, st));
  launch_modes_to_double((int)P, c->m_dev, c->mkd_dev, st);
  HIP_TRY(c, hipGetLastError());
  c->fixed_modes = true;
  return RBE_OK;
}

// One force evaluation of a single-system context on the state as given:
// charge checks, binning, sorted records, near field and Fourier part, Eq. 12,
// forces scattered back to the caller's order.
static int forces_body(rbe_ctx *c, const rbe_state *s, const int32_t *m, const double *w, uint64_t eval,
                       double *rho_out, hipStream_t st) {
  const int64_t n = s->n;
  launch_charge_check(c, n, s->q, st);
  {
    TScope ts(c, RBE_TK_BIN, st);
    launch_bin(c->bb, c->g, n, s->x, s->y, s->z, s->q, c->cell_start, c->perm, st);
  }
  {
    TScope ts(c, RBE_TK_REORDER, st);
    launch_gather_sorted(n, c->perm, s->x, s->y, s->z, s->q, s->id, c->g, c->srt, st);
  }
  WorkSet &o = c->ws[1];
  const int rc = eval_sorted(c, n, m, w, eval, rho_out, o.fx, o.fy, o.fz, st);
  if (rc != RBE_OK) return rc;
  if (c->pp.rbl && (c->p.terms & (RBE_TERM_LJ | RBE_TERM_COUL_REAL))) launch_sub_mean(n, c->mean, o.fx, o.fy, o.fz, st);
  launch_scatter_forces(n, c->perm, o.fx, o.fy, o.fz, s->fx, s->fy, s->fz, st);
  HIP_TRY(c, hipGetLastError());
  return RBE_OK;
}

extern "C" int rbe_forces(rbe_ctx *c, const rbe_state *s, const int32_t *m, const double *w, uint64_t eval,
                          double *rho_out, void *stream) {
  if (!c) return RBE_EINVAL;
  if (!state_ok(s, false)) return c->fail(RBE_EINVAL, "state has a null array");
  if (s->n < 1 || s->n > c->n_max)
    return c->fail(RBE_ERANGE, "n = %lld outside [1, n_max = %lld]", (long long)s->n, (long long)c->n_max);
  if ((m == nullptr) != (w == nullptr)) return c->fail(RBE_EINVAL, "m and w must both be given or both be NULL");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (c->batched()) return batch_forces(c, s, m, w, eval, rho_out, st);
  return forces_body(c, s, m, w, eval, rho_out, st);
}

extern "C" int rbe_energy(rbe_ctx *c, const rbe_state *s, const int32_t *m, const double *w, uint64_t eval,
                          double *u_out, double *rho_out, void *stream) {
  if (!c) return RBE_EINVAL;
  if (!s || !s->x || !s->y || !s->z || !s->q) return c->fail(RBE_EINVAL, "state has a null position or charge array");
  if (!u_out) return c->fail(RBE_EINVAL, "u_out is NULL");
  if ((s->vx == nullptr) != (s->vy == nullptr) || (s->vx == nullptr) != (s->vz == nullptr))
    return c->fail(RBE_EINVAL, "give all three velocity arrays or none");
  if (s->n < 1 || s->n > c->n_max)
    return c->fail(RBE_ERANGE, "n = %lld outside [1, n_max = %lld]", (long long)s->n, (long long)c->n_max);
  if ((m == nullptr) != (w == nullptr)) return c->fail(RBE_EINVAL, "m and w must both be given or both be NULL");
  if (c->batched()) return c->fail(RBE_EINVAL, "rbe_energy is not available on a batched context");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t n = s->n;
  launch_charge_check(c, n, s->q, st);
  const bool near = (c->p.terms & (RBE_TERM_LJ | RBE_TERM_COUL_REAL)) != 0;
  const bool fourier = (c->p.terms & RBE_TERM_FOURIER) != 0;
  launch_bin(c->bb, c->g, n, s->x, s->y, s->z, s->q, c->cell_start, c->perm, st);
  launch_gather_sorted(n, c->perm, s->x, s->y, s->z, s->q, s->id, c->g, c->srt, st);
  const int P = c->p.P;
  EnergyFinal fin{};
  if (fourier) {
    if (!m && c->fixed_modes) {
      m = c->m_dev;
      w = c->w_dev;
    } else if (!m) {
      launch_sample_modes(c->mt, c->cdf_dev, c->p.seed, eval, P, c->m_dev, c->w_dev, c->err, st);
      m = c->m_dev;
      w = c->w_dev;
    }
    launch_modes_to_double(P, m, c->fb.mkd, st);
    // structure factors always in FP64 here, whatever the context's precision
    const int32_t *nq = c->cell_start + c->g.ncell;
    launch_rho_partial(RBE_FP64, nq, n, P, c->srt.sq, c->fb, st);
    launch_rho_final(nq, P, c->fb, w, c->p.coulomb_k, rho_out, st);
    fin.w = w;
    fin.rho = c->fb.rho;
    fin.mkd = c->fb.mkd;
  }
  fin.P = P;
  for (int d = 0; d < 3; ++d) fin.L[d] = c->p.L[d];
  fin.alpha = c->p.alpha;
  fin.kc = c->p.coulomb_k;
  fin.self_coef = c->p.coulomb_k * std::sqrt(c->p.alpha / kPi);
  fin.half_mass = 0.5 * c->p.mass;
  fin.out = u_out;
  launch_energy(c->pp, 4.0 * c->p.lj_eps, n, c->srt, c->cell_start, near, s->q, s->vx, s->vy, s->vz, c->epart, fin,
                st);
  HIP_TRY(c, hipGetLastError());
  return RBE_OK;
}

// Reorder the working set through perm and pack the sorted records in one pass.
// With inv (random batch list), also the id -> slot map: inv[id] = k for ids
// inside [0, n) (the ids were validated by the call's first evaluation).
__global__ void __launch_bounds__(256) k_reorder_pack(int64_t n, const int32_t *__restrict__ perm, StateArrays in,
                                                      StateArrays out, Grid g, double4 *__restrict__ xq,
                                                      double4 *__restrict__ sq, int32_t *__restrict__ ids,
                                                      int32_t *__restrict__ inv) {
  const int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int j = perm[k];
  const double x = in.x[j], y = in.y[j], z = in.z[j], q = in.q[j];
  const int32_t id = in.id[j];
  if (inv && (uint32_t)id < (uint32_t)n) inv[id] = (int32_t)k;
  out.x[k] = x;
  out.y[k] = y;
  out.z[k] = z;
  out.vx[k] = in.vx[j];
  out.vy[k] = in.vy[j];
  out.vz[k] = in.vz[j];
  out.q[k] = q;
  out.id[k] = id;
  xq[k] = make_double4(x, y, z, q);
  if (q != 0.0) sq[k] = make_double4(x / g.L[0], y / g.L[1], z / g.L[2], q);
  ids[k] = id;
}

extern "C" int rbe_step(rbe_ctx *c, rbe_state *s, int32_t nsteps, uint64_t first_eval, void *stream) {
  if (!c) return RBE_EINVAL;
  if (!state_ok(s, true)) return c->fail(RBE_EINVAL, "state has a null array");
  if (s->n < 1 || s->n > c->n_max)
    return c->fail(RBE_ERANGE, "n = %lld outside [1, n_max = %lld]", (long long)s->n, (long long)c->n_max);
  if (nsteps < 0) return c->fail(RBE_EINVAL, "nsteps < 0");
  const bool nvt = c->p.nvt_tau > 0.0;
  if (nvt && !s->nh) return c->fail(RBE_EINVAL, "NVT needs the thermostat state s->nh");
  if (nvt && s->n < 2) return c->fail(RBE_EINVAL, "NVT needs at least two particles");
  if (nsteps == 0) return RBE_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  if (c->batched()) return batch_step(c, s, nsteps, first_eval, st);
  const int64_t n = s->n;
  launch_charge_check(c, n, s->q, st);
  // Step k advances X_k in place (kick, drift), reorders it into X_{k+1} and
  // evaluates the force there. X_0 is the caller's state and, with two or
  // more steps, so is X_nsteps: the last reorder writes the caller's arrays
  // directly; the steps between alternate between the two working sets.
  WorkSet S{s->x, s->y, s->z, s->vx, s->vy, s->vz, s->q, s->fx, s->fy, s->fz, s->id};
  auto next_set = [&](int32_t k) -> WorkSet * {
    if (nsteps >= 2 && k == nsteps - 1) return &S;
    return &c->ws[k % 2];
  };
  WorkSet *A = &S;
  const double h = 0.5 * c->p.dt / c->p.mass;
  const bool near = (c->p.terms & (RBE_TERM_LJ | RBE_TERM_COUL_REAL)) != 0;
  const bool fourier = (c->p.terms & RBE_TERM_FOURIER) != 0;
  const double *mean = (c->pp.rbl && near) ? c->mean : nullptr;
  NhParams nhp{};
  if (nvt) {
    nhp.dt = c->p.dt;
    nhp.nf = 3.0 * (double)n - 3.0;
    nhp.kT = c->p.nvt_kT;
    nhp.Q = nhp.nf * c->p.nvt_kT * c->p.nvt_tau * c->p.nvt_tau;
    nhp.mass = c->p.mass;
    // the first step's opening thermostat half on the caller's velocities
    TScope ts(c, RBE_TK_KICK, st);
    launch_nh(n, 0.0, nullptr, A->fx, A->fy, A->fz, A->vx, A->vy, A->vz, nhp, kNhStart, c->nh_part, s->nh,
              c->nh_scale, c->err, st);
  }
  for (int32_t k = 0; k < nsteps; ++k) {
    WorkSet *B = next_set(k);
    {
      // step 0 starts from the caller's forces; later NVE steps fuse the
      // previous step's second half-kick into this one's first half-kick and
      // drift (NVT steps cannot: the thermostat needs the kinetic energy
      // between the two half-kicks)
      // the drift also writes the binning keys and run slots of the new
      // positions (the keys pass of the counting sort, fused)
      TScope ts(c, RBE_TK_KICK_DRIFT, st);
      launch_bin_clear(c->bb, c->g, st);
      const BinKeyOut bk{A->q, c->bb.key, c->bb.slot, c->bb.count};
      if (k == 0 || nvt)
        launch_kick_drift(n, h, c->p.dt, c->g, nvt ? c->nh_scale : nullptr, A->fx, A->fy, A->fz, A->vx, A->vy, A->vz,
                          A->x, A->y, A->z, c->err, bk, st);
      else
        launch_kick_kick_drift(n, h, c->p.dt, c->g, mean, A->fx, A->fy, A->fz, A->vx, A->vy, A->vz, A->x, A->y,
                               A->z, c->err, bk, st);
    }
    {
      TScope ts(c, RBE_TK_BIN, st);
      launch_bin_place(c->bb, c->g, n, c->cell_start, c->perm, st);
    }
    {
      TScope ts(c, RBE_TK_REORDER, st);
      // from the second step on, the reorder also writes the id -> slot map
      // of the random batch list (the first step's evaluation validates ids)
      int32_t *inv = (k > 0 && c->pp.rbl && near) ? c->inv_id : nullptr;
      k_reorder_pack<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(n, c->perm, A->arrays(), B->arrays(), c->g,
                                                                   c->srt.xq, c->srt.sq, c->srt.id, inv);
    }
    const int64_t P = c->p.P;
    // a fixed table (rbe_set_modes) sits in slot 0 and is never redrawn
    const int ks = c->fixed_modes ? 0 : k % kSampleSteps;
    if (fourier && !c->fixed_modes && ks == 0) {
      // the mode samples of the next kSampleSteps evaluations in one launch
      TScope ts(c, RBE_TK_SAMPLE, st);
      launch_sample_modes(c->mt, c->cdf_dev, c->p.seed, first_eval + (uint64_t)k, (int)P, c->m_dev, c->w_dev, c->err,
                          st, std::min(kSampleSteps, nsteps - k), c->mkd_dev);
    }
    const int rc = eval_sorted(c, n, fourier ? c->m_dev + 3 * P * ks : nullptr, fourier ? c->w_dev + P * ks : nullptr,
                               first_eval + (uint64_t)k, nullptr, B->fx, B->fy, B->fz, st, k > 0,
                               fourier ? c->mkd_dev + 3 * P * ks : nullptr);
    if (rc != RBE_OK) return rc;
    if (nvt) {
      // second half-kick, the closing thermostat half of this step and, unless
      // this is the call's last step, the opening half of the next one
      TScope ts(c, RBE_TK_KICK, st);
      const bool last = k == nsteps - 1;
      launch_nh(n, h, mean, B->fx, B->fy, B->fz, B->vx, B->vy, B->vz, nhp, last ? kNhEnd : (kNhEnd | kNhStart),
                c->nh_part, s->nh, c->nh_scale, c->err, st);
      if (last) launch_scale_v(n, c->nh_scale, B->vx, B->vy, B->vz, st);
    } else if (k == nsteps - 1) {
      TScope ts(c, RBE_TK_KICK, st);
      launch_kick(n, h, mean, B->fx, B->fy, B->fz, B->vx, B->vy, B->vz, c->err, st);
    }
    A = B;
  }
  if (A != &S) {
    // a single step ends in a working set
    const double *src[10] = {A->x, A->y, A->z, A->vx, A->vy, A->vz, A->fx, A->fy, A->fz, A->q};
    double *dst[10] = {s->x, s->y, s->z, s->vx, s->vy, s->vz, s->fx, s->fy, s->fz, s->q};
    const int rc = copy_state(c, src, A->id, dst, s->id, n, st);
    if (rc != RBE_OK) return rc;
  }
  HIP_TRY(c, hipGetLastError());
  return RBE_OK;
}

extern "C" int rbe_sync_check(rbe_ctx *c, void *stream) {
  if (!c) return RBE_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  int flag = 0, bad_rep = -1;
  HIP_TRY(c, hipMemcpyAsync(&flag, c->err, sizeof flag, hipMemcpyDeviceToHost, st));
  if (c->batched()) HIP_TRY(c, hipMemcpyAsync(&bad_rep, c->bt.bad_rep, sizeof bad_rep, hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipStreamSynchronize(st));
  launch_fill_i32(c->err, 1, 0, st);
  HIP_TRY(c, hipStreamSynchronize(st));
  char who[48] = "";
  if (bad_rep >= 0) snprintf(who, sizeof who, " (replica %d)", bad_rep);
  if (flag & kErrNonFinite) return c->fail(RBE_ENONFINITE, "non-finite charge, velocity or force seen on the device%s", who);
  if (flag & kErrBadId) return c->fail(RBE_ERANGE, "a particle id lies outside [0, n)");
  if (flag & kErrSampler) return c->fail(RBE_EINVAL, "mode sampler rejected every attempt");
  if (flag & kErrGhostOverflow) return c->fail(RBE_ERANGE, "the ghost shell exceeded its capacity");
  if (flag & kErrBarrier) return c->fail(RBE_EDEVICE, "a grid barrier of the batched step timed out");
  if (flag & kErrNonNeutral) return c->fail(RBE_ENONNEUTRAL, "the charges do not sum to zero (Eq. 1)%s", who);
  if (flag & kErrTileOverflow)
    return c->fail(RBE_ERANGE, "a cell row of the near-field tiles exceeded the LDS staging (density far above the mean)");
  return RBE_OK;
}

extern "C" int rbe_set_counting(rbe_ctx *c, int enable) {
  if (!c) return RBE_EINVAL;
  c->counting = enable != 0;
  return RBE_OK;
}

extern "C" int rbe_get_counters(rbe_ctx *c, int64_t *counters, void *stream) {
  if (!c || !counters) return RBE_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  unsigned long long h[12];
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(c, hipMemcpyAsync(h, c->counters, sizeof h, hipMemcpyDeviceToHost, st));
  HIP_TRY(c, hipStreamSynchronize(st));
  for (int i = 0; i < 12; ++i) counters[i] = (int64_t)h[i];
  return RBE_OK;
}

extern "C" int rbe_set_timing(rbe_ctx *c, int enable) {
  if (!c) return RBE_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  Timer &t = c->tm;
  if (enable) {
    if (t.ev.empty()) {
      t.ev.resize(16384);
      // timing only: no system-scope release at each record (that release
      // writes back and invalidates the caches between the timed kernels)
      for (auto &e : t.ev) HIP_TRY(c, hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    }
    t.used = 0;
    t.kind.clear();
    t.count.clear();
    for (int k = 0; k < RBE_TIMING_KINDS; ++k) {
      t.ms[k] = 0.0;
      t.launches[k] = 0;
    }
  }
  t.on = enable != 0;
  return RBE_OK;
}

extern "C" int rbe_get_timing(rbe_ctx *c, double *ms_out, int64_t *launches_out, void *stream) {
  if (!c || !ms_out || !launches_out) return RBE_EINVAL;
  HIP_TRY(c, hipSetDevice(c->device));
  timer_flush(c, (hipStream_t)stream);
  for (int k = 0; k < RBE_TIMING_KINDS; ++k) {
    ms_out[k] = c->tm.ms[k];
    launches_out[k] = c->tm.launches[k];
  }
  return RBE_OK;
}

// ---------------------------------------------------------------------------
// rbe_forces without allocation: scratch in a file-scope device array
// ---------------------------------------------------------------------------
// Limits of the array (include/rbe.h): particles, keys of the cell grid (two
// species blocks), modes; structure-factor chunks at most kNoallocChunks.
constexpr int64_t kNoallocMaxN = RBE_NOALLOC_MAX_N;
constexpr int64_t kNoallocMaxKeys = RBE_NOALLOC_MAX_KEYS;
constexpr int kNoallocMaxP = RBE_NOALLOC_MAX_P;
constexpr int kNoallocChunks = 64;
constexpr size_t kNoallocBytes = (size_t)RBE_NOALLOC_SCRATCH_BYTES;

// The scratch of every rbe_forces_noalloc call on a device (each device holds
// its own copy until the process ends). Host code never uses this name as an
// address: the device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kNoallocBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
unsigned char *g_noalloc_ptr[kMaxDevices] = {};

// Bump carving of the scratch: every region starts on a 256-byte boundary.
struct Carve {
  unsigned char *base;
  size_t used, cap;
  bool ok = true;
  template <class T>
  T *take(int64_t count) {
    const size_t off = (used + 255) & ~(size_t)255;
    const size_t bytes = (size_t)(count < 1 ? 1 : count) * sizeof(T);
    if (off + bytes > cap) {
      ok = false;
      return nullptr;
    }
    used = off + bytes;
    return (T *)(base + off);
  }
};
}  // namespace

// Device address of this device's scratch, resolved once per device with the
// device current; the FP64 turn table is written once at the start of it (no
// call overwrites that region).
static unsigned char *noalloc_scratch(int device, std::string *why) {
  if (device < 0 || device >= kMaxDevices) {
    *why = "device index out of range";
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (g_noalloc_ptr[device]) return g_noalloc_ptr[device];
  void *ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) {
    *why = std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e);
    return nullptr;
  }
  static double2 turn_host[kTurnTableEntries];
  static std::once_flag turn_once;
  std::call_once(turn_once, [] { fill_turn_table(turn_host, kTurnTableEntries); });
  if (hipMemcpy(ptr, turn_host, sizeof turn_host, hipMemcpyHostToDevice) != hipSuccess) {
    *why = "copy of the turn table into the scratch array failed";
    return nullptr;
  }
  g_noalloc_ptr[device] = (unsigned char *)ptr;
  return g_noalloc_ptr[device];
}

// status_out[0] = the rbe_status of the device-side checks of this call.
__global__ void k_noalloc_status(const int *err, int32_t *status_out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int f = *err;
  int st = RBE_OK;
  if (f & kErrNonNeutral) st = RBE_ENONNEUTRAL;
  if (f & (kErrGhostOverflow | kErrTileOverflow)) st = RBE_ERANGE;
  if (f & kErrBadId) st = RBE_ERANGE;
  if (f & kErrNonFinite) st = RBE_ENONFINITE;
  *status_out = st;
}

extern "C" int rbe_forces_noalloc(const rbe_params *p, const rbe_state *s, const int32_t *m, const double *w,
                                  uint64_t eval, double *rho_out, int32_t *status_out, void *stream) {
  if (!p) return create_fail(RBE_EINVAL, "params is NULL");
  if (!state_ok(s, false)) return create_fail(RBE_EINVAL, "state has a null array");
  if (!m || !w) return create_fail(RBE_EINVAL, "rbe_forces_noalloc needs the mode sample m, w");
  if (s->n < 1 || s->n > kNoallocMaxN) return create_fail(RBE_ERANGE, "n outside [1, RBE_NOALLOC_MAX_N]");
  if (p->P > kNoallocMaxP) return create_fail(RBE_ERANGE, "P exceeds RBE_NOALLOC_MAX_P");
  if (p->ghost_width > 0) return create_fail(RBE_EINVAL, "rbe_forces_noalloc has no ghost shell");
  std::string why;
  int rc = validate_params(p, &why);
  if (rc != RBE_OK) return create_fail(rc, why.c_str());
  int device = 0;
  if (hipGetDevice(&device) != hipSuccess) return create_fail(RBE_EDEVICE, "hipGetDevice failed");
  unsigned char *base = noalloc_scratch(device, &why);
  if (!base) return create_fail(RBE_EDEVICE, why.c_str());

  rbe_ctx c;  // host-side description only; every device region is carved from the scratch
  c.device = device;
  rc = ctx_geometry(&c, p, s->n, &why);
  if (rc != RBE_OK) return create_fail(rc, why.c_str());
  const int64_t n = s->n;
  const int64_t nkeys = 2 * (int64_t)c.g.ncell;
  if (nkeys > kNoallocMaxKeys) return create_fail(RBE_ERANGE, "the cell grid exceeds RBE_NOALLOC_MAX_KEYS keys");
  const int P = c.p.P;
  Carve cv{base, 0, kNoallocBytes};
  c.fb.turn_tab = cv.take<double2>(kTurnTableEntries);  // written once per device
  c.bb.key = cv.take<int32_t>(n);
  c.bb.slot = cv.take<int32_t>(n);
  c.bb.tmp = cv.take<int32_t>(n);
  c.bb.count = cv.take<int32_t>(nkeys);
  c.bb.scan_tmp = cv.take<int32_t>(scan_tiles(nkeys));
  c.cell_start = cv.take<int32_t>(nkeys + 1);
  c.perm = cv.take<int32_t>(n);
  c.inv_id = cv.take<int32_t>(n);
  c.srt.xq = cv.take<double4>(n + kScanPad);
  c.srt.sq = cv.take<double4>(n);
  c.srt.id = cv.take<int32_t>(n + kScanPad);
  c.ws[1].fx = cv.take<double>(n);
  c.ws[1].fy = cv.take<double>(n);
  c.ws[1].fz = cv.take<double>(n);
  c.fb.nchunk_max = kNoallocChunks;
  c.fb.mkd = cv.take<double>(3 * (int64_t)P);
  c.fb.part = cv.take<double2>((int64_t)kNoallocChunks * P);
  c.fb.rho = cv.take<double>(2 * (int64_t)P);
  c.fb.modes = cv.take<GatherMode>(P);
  c.fb.gpart = nullptr;  // no mode split in the scratch-only form
  c.mean_part = cv.take<double>(3 * (int64_t)mean_blocks(n) + 3);
  c.mean = cv.take<double>(3);
  c.err = cv.take<int>(1);
  c.qstats = cv.take<double>(2);
  if (!cv.ok) return create_fail(RBE_ERANGE, "the problem does not fit the scratch array");
  hipStream_t st = (hipStream_t)stream;
  launch_fill_i32(c.err, 1, 0, st);  // the array keeps the previous call's flag
  rc = forces_body(&c, s, m, w, eval, rho_out, st);
  if (rc != RBE_OK) return create_fail(rc, c.last_error.c_str());
  if (status_out) k_noalloc_status<<<1, 64, 0, st>>>(c.err, status_out);
  if (hipGetLastError() != hipSuccess) return create_fail(RBE_EDEVICE, "a launch failed");
  return RBE_OK;
}
