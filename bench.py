"""Throughput of the RBE nonbonded force + velocity-Verlet step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--prec fp64|fp32c]

A step is one pass of the whole hot path over the system: half-kick + drift
+ wrap, cell binning and reorder, ghost shell (where the workload has one),
mode sample, near field (with the core-shell random batch list where the
workload has one), structure factors, Fourier gather and the second
half-kick. Inputs are synthetic (seeded generator) and resident in HBM before
the timed region. Prints one JSON line.

The default workload, "headline", is the metric's own comparison: the
FP32-compensated form on one GPU's 64M-particle subdomain with its 6-sigma
ghost shell (P = 1000), beside the plain FP64 GPU path on the same system,
and the batched form on 256 replicas beside its FP64 forms and per-replica
loops. `value` is the FP32C particle-steps/s of the subdomain (median of the
repeats, no per-kernel events in the timed region). Every form carries its
RMS relative force error against the FP64 CPU oracle, per term and total.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s RBE nonbonded force, FP32-comp & batched vs FP64, ≤1e-5 err"

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit (FMA = 2 flops; a special function counts 1),
# counted on the pair terms inside the cutoffs only (candidates outside, the
# shell walk and ranking of the random batch list are overhead):
#   near field: per Coulomb pair term 27 flops, per LJ pair term 22 flops
#   structure factor: 13 flops per (charged particle, mode)
#   gather: 18 flops per (charged particle, mode)
FLOPS_COUL_PAIR = 27
FLOPS_LJ_PAIR = 22
FLOPS_RHO_IK = 13
FLOPS_GATHER_IK = 18
# HBM bytes per particle of the streaming kernels
BYTES_KICK_DRIFT = 120   # read f (24) v (24) x (24), write v (24) x (24)
BYTES_KICK = 96          # read f (24) v (24), write v (24) f (24)

# cell edges picked by paper_2609_02694_amd.tune on MI355X: (edge along y and z,
# x cells per y/z cell edge)
DEFAULT_NCELL_H = {"plain3k": 3.0, "electrolyte1m": 3.0, "ions8m": 4.0, "subdomain64m": 2.5, "replica": 2.5,
                   "ljelectrolyte": 8.2}
DEFAULT_XSPLIT = {"plain3k": 1, "electrolyte1m": 6, "ions8m": 6, "subdomain64m": 4, "replica": 3,
                  "ljelectrolyte": 4}

# Particles of the same-physics reduced system on which every row and term is
# compared with the oracle (the oracle's structure factors of the full
# subdomain would take about a minute of host time).
EPS_REDUCED_N = 200_000
EPS_SAMPLED_ROWS = 256


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--repeats", type=int, default=5, help="timed repeats of K steps (median, min, max)")
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "plain3k", "electrolyte1m", "ions8m", "subdomain64m", "replica256",
                             "ljelectrolyte"])
    ap.add_argument("--compare-steps", type=int, default=None,
                    help="steps of each comparison form (default: --steps); 0 skips them")
    ap.add_argument("--edge", type=float, default=None, help="cell edge (along y and z; replica256: all axes)")
    ap.add_argument("--xsplit", type=int, default=None, help="x cells per y/z cell edge")
    ap.add_argument("--tune", action="store_true",
                    help="pick the grid with the autotuner (cached in --tune-cache) instead of the defaults")
    ap.add_argument("--tune-cache", default=os.environ.get("RBE_TUNE_CACHE", os.path.join(ROOT, ".tune_cache.json")))
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32c"])
    ap.add_argument("--n", type=int, default=None, help="override the particle count (same density)")
    ap.add_argument("--rbl-shell", default=None, choices=["all", "charged"],
                    help="shell population of the random batch list (default: the preset's, i.e. all)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-eps", action="store_true", help="skip the force-error comparison with the oracle")
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel HIP event pass")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scale of the HBM byte counters)")
    ap.add_argument("--calibrate-valu", action="store_true",
                    help="only run the vector-ALU issue-rate probe (include/rbe_probe.h), each mix twice")
    return ap.parse_args()


def log(msg):
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def calibrate_copy(mib):
    """Five plain device-to-device copies of `mib` MiB: the HBM byte counters of
    one such copy should read `mib` MiB fetched and `mib` MiB written."""
    import torch

    n = mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(5):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibrate_copy_mib": mib, "bytes_per_copy": 2 * n * 8}), flush=True)


def calibrate_valu(rbe):
    """The vector-ALU issue-rate probe, each instruction mix twice (the first
    launch warms up): the SIMD cycles one wave64 instruction of the mix takes
    follow from rocprofv3's SQ_INSTS_VALU and GRBM_GUI_ACTIVE of the second."""
    blocks, iters = 4096, 4000
    for kind in rbe.PROBE_KINDS:
        ms = [rbe.probe_valu(kind, blocks, iters) for _ in range(2)]
        print(json.dumps({"calibrate_valu": kind, "blocks": blocks, "iters": iters, "ms": ms[1]}), flush=True)


# ---------------------------------------------------------------------------
# timing
# ---------------------------------------------------------------------------
def timed_steps(ctx, st, K, first_eval, stream):
    """Wall time of exactly K steps, synchronized on both sides (HIP events on
    the launch stream alongside)."""
    import torch

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(st, K, first_eval)
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    return w1 - w0, ev0.elapsed_time(ev1) / 1000.0


def repeat_stats(n, K, walls):
    ms = [1000.0 * w / K for w in walls]
    med = statistics.median(ms)
    return {"repeats": len(ms), "ms_per_step": [round(v, 4) for v in ms], "median_ms": med, "min_ms": min(ms),
            "max_ms": max(ms), "particle_steps_per_s": n / (med * 1e-3)}


def kernel_table(kt):
    return {k: {"total_ms": round(v[0], 4), "launches": v[1], "avg_us": round(1000 * v[0] / v[1], 3)}
            for k, v in kt.items() if v[1] > 0}


def run_form(rbe, p, s, prec, grid, K, W, repeats, timing=True, counting=True):
    """One precision form of one system: counting pass, initial force, W
    warmup steps, `repeats` timed runs of K steps, then a separate pass of K
    steps with per-kernel HIP events. Returns (stats, kernels, counts)."""
    import torch

    n = p["n"]
    ctx = rbe.Context(rbe.params_from_preset(p, prec=prec, ncell=grid), n)
    st = rbe.Particles.from_numpy(s)
    if p.get("nvt_tau", 0.0) > 0:
        st.nh = torch.zeros(2, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    cnt = None
    if counting:
        ctx.set_counting(True)
        ctx.forces(st, None, None, 0)
        cnt = ctx.counters()
        ctx.set_counting(False)
    ctx.forces(st, None, None, 0)
    ev = 1
    if W > 0:
        ctx.step(st, W, ev)
        ev += W
    torch.cuda.synchronize()
    ctx.sync_check()
    walls, evs = [], []
    for _ in range(repeats):
        w, e = timed_steps(ctx, st, K, ev, stream)
        ev += K
        walls.append(w)
        evs.append(e)
    ctx.sync_check()
    stats = repeat_stats(n, K, walls)
    stats["event_ms_per_step_median"] = 1000.0 * statistics.median(evs) / K
    kernels = {}
    if timing:
        ctx.set_timing(True)
        ctx.step(st, K, ev)
        kernels = kernel_table(ctx.timing())
        ctx.set_timing(False)
        ctx.sync_check()
    ctx.close()
    del st
    torch.cuda.empty_cache()
    return stats, kernels, cnt


# ---------------------------------------------------------------------------
# force error against the oracle
# ---------------------------------------------------------------------------
TERM_NAMES = ("lj", "coul_real", "fourier")


def rel_err(a, b):
    import numpy as np

    nb = float(np.linalg.norm(b))
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def gpu_term_forces(rbe, p, s, prec, grid, terms, m, w, ev=0):
    import numpy as np
    import torch

    ctx = rbe.Context(rbe.params_from_preset(p, prec=prec, terms=terms, ncell=grid), p["n"])
    st = rbe.Particles.from_numpy(s)
    md = torch.as_tensor(np.ascontiguousarray(m, np.int32).ravel()).cuda()
    wd = torch.as_tensor(np.ascontiguousarray(w, np.float64)).cuda()
    ctx.forces(st, md, wd, ev)
    torch.cuda.synchronize()
    ctx.sync_check()
    F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
    ctx.close()
    del st
    torch.cuda.empty_cache()
    return F


def eps_every_row(rbe, p, s, grid, precs, ev=0):
    """RMS relative error of every row, per term and total, against the
    oracle's forces of the same system and mode sample (random batch list
    and Eq. 12 where the system has them)."""
    import oracle

    m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
    osys = oracle.sys_from_preset(p)
    ref = oracle.total_force(s["x"], s["y"], s["z"], s["q"], s["id"], osys, m, w, seed=p["seed"], ev=ev,
                             cells=True if p["n"] > 20000 else None)
    terms = {"lj": ref["lj"], "coul_real": ref["coul"], "fourier": ref["fourier"]}
    if p.get("r_core", 0.0) > 0:
        # each near-field term alone carries its own Eq. 12 mean
        for t in ("lj", "coul_real"):
            terms[t] = oracle.mean_correct(terms[t])[0]
    out = {}
    for prec in precs:
        name = "fp64" if prec == rbe.FP64 else "fp32c"
        e = {}
        for t, mask in zip(TERM_NAMES, (rbe.TERM_LJ, rbe.TERM_COUL_REAL, rbe.TERM_FOURIER)):
            F = gpu_term_forces(rbe, p, s, prec, grid, mask, m, w, ev)
            e[t] = rel_err(F, terms[t])
        F = gpu_term_forces(rbe, p, s, prec, grid, rbe.TERM_ALL, m, w, ev)
        e["total"] = rel_err(F, ref["F"])
        e["max_row_over_rms"] = float(abs(F - ref["F"]).max() / ((ref["F"] ** 2).sum() / len(F)) ** 0.5)
        out[name] = e
    return out


def sampled_rows(s, nrows, seed=7):
    """Rows to compare at full size: charged and neutral particles, the first
    and last particles, and particles close to a box face."""
    import numpy as np

    rng = np.random.default_rng(seed)
    n = len(s["x"])
    q = s["q"]
    charged = np.flatnonzero(q != 0)
    neutral = np.flatnonzero(q == 0)
    L = float(s["L"][0])
    face = np.flatnonzero(np.minimum(s["x"], L - s["x"]) < 0.05)
    k = nrows // 4
    parts = [rng.choice(charged, min(k, len(charged)), replace=False),
             rng.choice(neutral, min(k, len(neutral)), replace=False) if len(neutral) else np.zeros(0, np.int64),
             rng.choice(face, min(k, len(face)), replace=False) if len(face) else np.zeros(0, np.int64),
             np.arange(max(0, n - k // 2), n), np.arange(0, min(n, k // 2))]
    return np.unique(np.concatenate(parts).astype(np.int64))


def eps_sampled_near(rbe, p, s, grid, precs, nrows, ev=0):
    """Full size: RMS relative error of the near field (LJ + screened Coulomb)
    on sampled rows against the oracle's per-row sums (no random batch list
    in the workloads this is used on, so rows are independent)."""
    import oracle

    idx = sampled_rows(s, nrows)
    osys = oracle.sys_from_preset(p)
    ref = oracle.real_force(s["x"], s["y"], s["z"], s["q"], s["id"], osys, seed=p["seed"], ev=ev, idx=idx, cells=True)
    m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
    out = {"rows": int(len(idx))}
    for prec in precs:
        F = gpu_term_forces(rbe, p, s, prec, grid, rbe.TERM_LJ | rbe.TERM_COUL_REAL, m, w, ev)
        out["fp64" if prec == rbe.FP64 else "fp32c"] = rel_err(F[idx], ref)
    return out


# ---------------------------------------------------------------------------
# rooflines (algorithmic accounting: in-cutoff pair terms only)
# ---------------------------------------------------------------------------
# Fourier kernels, issue-slot model backed by rocprofv3 SQ counters
# (profiles/step_subdomain64m_fp32c.md): the hardware sine and cosine of the
# FP32C kernels are counted apart (SQ_INSTS_VALU_TRANS_F32) because they issue
# on the transcendental pipe beside the other VALU work, so the bound used is
# the VALU issue rate, 256 CU x 64 lanes x 2.4 GHz = 39.3 T lane-slots/s.
# Algorithmic lane slots per (charged particle, mode): the FP64 phase (3
# multiply-adds, rint, subtract: 5) and its conversion to FP32 (1), then 2
# FMAs (structure factor) or 5 (gather: g = a cos - b sin, then g m
# accumulated); the two transcendentals are reported as a rate of their own.
PEAK_LANE_SLOTS_T = 256 * 64 * 2.4e9 / 1e12
SLOTS_RHO_IK = 5 + 1 + 2
SLOTS_GATHER_IK = 5 + 1 + 5


def pair_flops(c):
    """Algorithmic flops of one near-field launch from its counters
    (coul_pairs, lj_pairs, candidates, shell_members)."""
    return FLOPS_COUL_PAIR * c[0] + FLOPS_LJ_PAIR * c[1]


def kernel_roofline(name, kernels, cnt, nq, p, prec):
    """Roofline entry of one timed kernel kind (None if no model applies)."""
    if name not in kernels:
        return None
    avg_s = kernels[name]["avg_us"] * 1e-6
    peak_alu = PEAK_FP64_TFLOPS if prec == 0 else PEAK_FP32_TFLOPS
    n, P = p["n"], p["P"]
    if name.startswith("pair") and cnt and name in cnt:
        c = cnt[name]
        work = pair_flops(c)
        ach = work / avg_s / 1e12
        r = dict(kernel=name, bound="alu", achieved=ach, peak=peak_alu, unit="TFLOP/s", frac=ach / peak_alu,
                 work_per_launch=work, pairs_per_launch=int(c[0] + c[1]), candidates_per_launch=int(c[2]))
        if c[3]:
            # walk, classification and ranking of the shell of Eq. 10-11:
            # overhead, reported as its own rate
            r["shell_members_per_s"] = c[3] / avg_s
        return r
    if name in ("rho_partial", "gather"):
        per = SLOTS_RHO_IK if name == "rho_partial" else SLOTS_GATHER_IK
        work = per * nq * P
        ach = work / avg_s / 1e12
        return dict(kernel=name, bound="alu", achieved=ach, peak=PEAK_LANE_SLOTS_T, unit="Tslot/s",
                    frac=ach / PEAK_LANE_SLOTS_T, work_per_launch=work,
                    model="non-transcendental VALU issue slots; sin/cos on the transcendental pipe",
                    transcendentals_per_s=2 * nq * P / avg_s)
    per_bytes = {"kick_drift": BYTES_KICK_DRIFT, "kick": BYTES_KICK}.get(name)
    if per_bytes is None:
        return None
    ach = per_bytes * n / avg_s / 1e9
    return dict(kernel=name, bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS,
                work_per_launch=per_bytes * n)


def measured_traffic(workload, name, grid=None, form=None):
    """HBM bytes per launch of a kernel kind from the committed rocprofv3 counter
    runs (profiles/traffic.json), or None when the kernel sources, the form
    or the cell grid differ from the counted run."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    recs = json.load(open(path))
    # a record per workload and form ("subdomain64m:fp64"), or one for the
    # workload whose "form" names the form it was counted on
    d = recs.get(f"{workload}:{form}") if form is not None else None
    d = d or recs.get(workload)
    if not d or name not in d.get("kinds", {}):
        return None
    if form is not None and d.get("form") not in (None, form):
        return None
    h = hashlib.sha256()
    for f in d["files"]:
        fp = os.path.join(ROOT, f)
        if not os.path.exists(fp):
            return None
        h.update(open(fp, "rb").read())
    if h.hexdigest() != d["source_sha256"]:
        return None
    if grid is not None and d.get("grid") != grid:
        return None
    t = d["kinds"][name]
    return t["read_bytes"] + t["write_bytes"]


def roofline(kernels, cnt, nq, p, prec, workload=None, grid=None, form=None):
    """Roofline figure of the dominant kernel (largest summed time), and of every kind with a model."""
    if not kernels:
        return None, {}
    every = {k: kernel_roofline(k, kernels, cnt, nq, p, prec) for k in kernels}
    every = {k: v for k, v in every.items() if v}
    name = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dom = every.get(name) or dict(kernel=name, bound="alu", achieved=None, peak=None, unit=None, frac=None)
    dom = dict(dom)
    dom["traffic"] = measured_traffic(workload, name, grid, form) if workload else None
    # counted HBM bytes per launch over the live average duration, against the
    # HBM peak (shown for every kind, whatever bounds it)
    for k, r in [(name, dom)] + list(every.items()):
        t = dom["traffic"] if k == name else (measured_traffic(workload, k, grid, form) if workload else None)
        if t and kernels[k]["avg_us"] > 0:
            r["hbm_gbps"] = t / (kernels[k]["avg_us"] * 1e-6) / 1e9
            r["hbm_frac"] = r["hbm_gbps"] / PEAK_HBM_GBS
    return dom, every


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------
def cpu_info():
    """CPU model, sockets and physical cores of this host (lscpu), and the
    oracle's thread count."""
    import oracle

    info = {"model": None, "sockets": None, "physical_cores": None, "logical_cpus": os.cpu_count(),
            "oracle_threads": oracle.num_threads()}
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        kv = {}
        for ln in out.splitlines():
            if ":" in ln:
                k, v = ln.split(":", 1)
                kv[k.strip()] = v.strip()
        info["model"] = kv.get("Model name")
        if kv.get("Socket(s)", "").isdigit():
            info["sockets"] = int(kv["Socket(s)"])
        if kv.get("Core(s) per socket", "").isdigit() and info["sockets"]:
            info["physical_cores"] = info["sockets"] * int(kv["Core(s) per socket"])
    except (OSError, subprocess.SubprocessError):
        pass
    if not info["model"]:
        try:
            with open("/proc/cpuinfo") as f:
                info["model"] = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
        except OSError:
            pass
    return info


def oracle_vv_step(p, s, ev=1):
    """One velocity-Verlet step of the oracle (half-kick from zero force,
    drift + wrap, force evaluation ev with its mode sample and batch list,
    half-kick): the step the GPU times, on the host."""
    import numpy as np

    import oracle

    osys = oracle.sys_from_preset(p)
    m, w = oracle.sample_k(p["seed"], ev, p["L"], p["alpha"], p["P"])
    r = np.stack([s["x"], s["y"], s["z"]], axis=1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)
    v = oracle.kick(np.zeros_like(r), v, p["dt"] / 2)
    r = oracle.drift_wrap(r, v, p["dt"], p["L"])
    F = oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, m, w, seed=p["seed"], ev=ev,
                           components=False, cells=True if p["n"] > 20000 else None)["F"]
    return oracle.kick(F, v, p["dt"] / 2)


def oracle_plain3k_seconds():
    """The small parity workload in full (one force evaluation and ten
    velocity-Verlet steps) on one thread and on all threads."""
    import gen
    import oracle

    p = gen.preset("plain3k")
    s = gen.make_system(p)
    nt = oracle.num_threads()
    out = {}
    for k in (1, nt):
        oracle.set_num_threads(k)
        t0 = time.perf_counter()
        for ev in range(11):
            oracle_vv_step(p, s, ev)
        out[f"threads_{k}"] = round(time.perf_counter() - t0, 3)
    oracle.set_num_threads(nt)
    return out


def cpu_baseline_sample(p, s, label):
    """The oracle on one velocity-Verlet step of a bounded sample of the
    workload (a system of the same composition, whose cost per particle is
    the workload's), on all host threads; particle-steps/s extrapolated."""
    import oracle

    t0 = time.perf_counter()
    oracle_vv_step(p, s)
    dt = time.perf_counter() - t0
    return {"value": p["n"] / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": label, "seconds": round(dt, 2)}


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def grid_of(p, name, a):
    h = a.edge or DEFAULT_NCELL_H.get(name, 3.0)
    nc = max(1, int(p["L"] // h))
    return (nc * (a.xsplit or DEFAULT_XSPLIT.get(name, 1)), nc, nc)


def bench_single(a, rbe, workload, prec_name, repeats, with_other=True, with_eps=True, with_cpu=True):
    """One system in one precision form, with the other form beside it."""
    import numpy as np

    import gen

    p = gen.preset(workload, n=a.n)
    if a.rbl_shell:
        if a.rbl_shell == "charged" and not p.get("r_core", 0.0) > 0.0:
            print(f"--rbl-shell charged needs a workload with the random batch list ({workload} has none)",
                  file=sys.stderr)
            sys.exit(2)
        p["rbl_shell"] = 1 if a.rbl_shell == "charged" else 0
    prec = rbe.FP64 if prec_name == "fp64" else rbe.FP32C
    grid = grid_of(p, workload, a)
    tuned = None
    t0 = time.time()
    s = gen.make_system(p)
    t_gen = time.time() - t0
    log(f"{workload}: generated {p['n']} particles in {t_gen:.1f} s, grid {grid}")
    if a.tune:
        from paper_2609_02694_amd import tune
        t1 = time.time()
        (nx, nc, _), hit = tune.tune_grid_cached(p, s, prec, a.tune_cache, steps=10)
        grid = (nx, nc, nc)
        tuned = dict(cache_hit=hit, seconds=round(time.time() - t1, 1))
    K, W = a.steps, a.warmup
    stats, kernels, cnt = run_form(rbe, p, s, prec, grid, K, W, repeats, timing=not a.no_timing)
    log(f"{workload} {prec_name}: {stats['median_ms']:.3f} ms/step")
    nq = int(np.count_nonzero(s["q"]))
    roof, roofs = roofline(kernels, cnt, nq, p, prec, workload=workload, grid=list(grid), form=prec_name)
    forms = {prec_name: stats}
    Kc = K if a.compare_steps is None else a.compare_steps
    if with_other and Kc > 0:
        other = rbe.FP32C if prec == rbe.FP64 else rbe.FP64
        oname = "fp32c" if other == rbe.FP32C else "fp64"
        ost, okern, ocnt = run_form(rbe, p, s, other, grid, Kc, min(W, 3), max(1, repeats // 2 + 1),
                                    timing=not a.no_timing, counting=True)
        log(f"{workload} {oname}: {ost['median_ms']:.3f} ms/step")
        oroof, _ = roofline(okern, ocnt, nq, p, other, workload=workload, grid=list(grid), form=oname)
        ost["roofline"] = oroof
        forms[oname] = ost
    eps = None
    if with_eps and not a.no_eps:
        t1 = time.time()
        precs = [rbe.FP32C, rbe.FP64] if with_other else [prec]
        if p["n"] <= 1_000_000:
            eps = {"every_row": eps_every_row(rbe, p, s, grid, precs), "system": f"the full {p['n']}-particle system"}
        else:
            # every row of a same-physics reduced system, and sampled rows of the full one
            pr = gen.preset(workload, n=EPS_REDUCED_N)
            sr = gen.make_system(pr)
            eps = {"every_row": eps_every_row(rbe, pr, sr, grid_of(pr, workload, a), precs),
                   "system": f"every row: {EPS_REDUCED_N} particles at the workload's density, composition, "
                             f"cutoffs, P and ghost shell; sampled: {EPS_SAMPLED_ROWS} rows of the full system "
                             "(near field)",
                   "sampled_full_near_field": eps_sampled_near(rbe, p, s, grid, precs, EPS_SAMPLED_ROWS)}
        eps["seconds"] = round(time.time() - t1, 1)
        log(f"{workload}: force errors {eps}")
    out = {
        "value": stats["particle_steps_per_s"],
        "ms_per_step": stats["median_ms"],
        "dtype": "f64" if prec == rbe.FP64 else "f32+f64",
        "config": {"workload": workload, "n": p["n"], "n_charged": nq, "L": round(p["L"], 4), "alpha": p["alpha"],
                   "r_coul": p["r_coul"], "r_lj": p["r_lj"], "r_core": p["r_core"], "p_shell": p["p_shell"],
                   "P": p["P"], "dt": p["dt"], "ghost_width": p.get("ghost", 0.0), "form": prec_name,
                   "ncell": list(grid), "tuned": tuned,
                   "ensemble": "NVT" if p.get("nvt_tau", 0.0) > 0 else "NVE",
                   "rbl_shell": "charged" if p.get("rbl_shell", 0) else "all", "parallelism": "single GPU"},
        "timing": {k: v for k, v in stats.items() if k != "particle_steps_per_s"},
        "forms": {k: {"particle_steps_per_s": v["particle_steps_per_s"], "median_ms": v["median_ms"],
                      "min_ms": v["min_ms"], "max_ms": v["max_ms"], "repeats": v["repeats"],
                      **({"roofline": v["roofline"]} if "roofline" in v else {})} for k, v in forms.items()},
        "kernels": kernels,
        "counts_per_eval": {k: dict(zip(("coul_pairs", "lj_pairs", "candidates", "shell_members"), v))
                            for k, v in (cnt or {}).items()},
        "roofline": roof,
        "rooflines": roofs,
        "epsilon": eps,
        "gen_s": round(t_gen, 2),
    }
    if len(forms) == 2:
        f32 = forms.get("fp32c", {}).get("particle_steps_per_s")
        f64 = forms.get("fp64", {}).get("particle_steps_per_s")
        if f32 and f64:
            out["fp32c_over_fp64"] = f32 / f64
    if with_cpu and not a.no_cpu_baseline:
        t1 = time.time()
        if p["n"] <= 1_000_000:
            out["cpu_baseline"] = cpu_baseline_sample(p, s, f"one velocity-Verlet step of the full "
                                                            f"{p['n']}-particle system")
        else:
            pr = gen.preset(workload, n=EPS_REDUCED_N)
            sr = gen.make_system(pr)
            out["cpu_baseline"] = cpu_baseline_sample(
                pr, sr, f"one velocity-Verlet step of a {EPS_REDUCED_N}-particle system of the workload's density, "
                        "composition, cutoffs and P (the oracle's cost grows linearly in N at fixed P); "
                        f"extrapolated to the {p['n']}-particle workload")
        out["cpu_baseline"]["cpu"] = cpu_info()
        out["cpu_baseline"]["plain3k_full_s"] = oracle_plain3k_seconds()
        log(f"{workload}: cpu baseline {time.time() - t1:.1f} s")
    return out


def bench_batch(a, rbe, repeats, with_eps=True, with_cpu=True):
    """256 replicas of uneven size advanced together by the batched form."""
    import numpy as np
    import torch

    import gen
    from paper_2609_02694_amd import tune

    prec_name = a.prec or "fp32c"
    prec = rbe.FP64 if prec_name == "fp64" else rbe.FP32C
    t0 = time.time()
    sizes = gen.replica_sizes(256)
    reps, cat, off = gen.replica_batch(sizes)
    t_gen = time.time() - t0
    ntot = int(off[-1])
    log(f"replica256: generated {ntot} particles in {t_gen:.1f} s")
    edge = a.edge or DEFAULT_NCELL_H["replica"]
    xsplit = a.xsplit or DEFAULT_XSPLIT["replica"]
    tuned = None
    if a.tune:
        t1 = time.time()
        (edge, xsplit), hit = tune.tune_batch_cached(reps, cat, off, prec, a.tune_cache, steps=5)
        tuned = dict(cache_hit=hit, seconds=round(time.time() - t1, 1))
    K, W = a.steps, a.warmup
    stream = torch.cuda.current_stream()

    def batched(pr, reps_n, timing):
        ctx = rbe.Context.batch(tune.batch_params(reps, edge, pr, xsplit), off)
        st = rbe.Particles.from_numpy(cat)
        ctx.forces(st, None, None, 0)
        ev = 1
        if W > 0:
            ctx.step(st, W, ev)
            ev += W
        torch.cuda.synchronize()
        ctx.sync_check()
        walls = []
        for _ in range(reps_n):
            w, _ = timed_steps(ctx, st, K, ev, stream)
            ev += K
            walls.append(w)
        ctx.sync_check()
        kern = {}
        if timing:
            ctx.set_timing(True)
            ctx.step(st, K, ev)
            kern = kernel_table(ctx.timing())
            ctx.set_timing(False)
            ctx.sync_check()
        ctx.close()
        return repeat_stats(ntot, K, walls), kern

    stats, kernels = batched(prec, repeats, not a.no_timing)
    log(f"replica256 batched {prec_name}: {stats['median_ms']:.3f} ms/step")
    forms = {f"batched_{prec_name}": stats}
    Kc = K if a.compare_steps is None else a.compare_steps

    def loop_rate(pr, steps):
        """particle-steps/s of a loop of single-system contexts (and, for
        FP64, the pair counts of one evaluation)."""
        ctxs, sts = [], []
        for (p, s) in reps:
            n = max(1, int(p["L"] // edge))
            ctxs.append(rbe.Context(rbe.params_from_preset(p, prec=pr, ncell=(xsplit * n, n, n),
                                                           seed=p["stream_seed"]), p["n"]))
            sts.append(rbe.Particles.from_numpy(s))
        for c, s_ in zip(ctxs, sts):
            c.forces(s_, None, None, 0)
            c.step(s_, 2, 1)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for c, s_ in zip(ctxs, sts):
            c.step(s_, steps, 3)
        torch.cuda.synchronize()
        rate = ntot * steps / (time.perf_counter() - t)
        counts = None
        if pr == rbe.FP64:
            counts = [0, 0, 0, 0]
            for c, s_ in zip(ctxs, sts):
                c.set_counting(True)
                c.forces(s_, None, None, 0)
                for v in c.counters().values():
                    for i in range(4):
                        counts[i] += v[i]
        for c in ctxs:
            c.sync_check()
            c.close()
        return rate, counts

    v64_loop, counts = loop_rate(rbe.FP64, max(2, Kc // 2) if Kc > 0 else 2)
    if Kc > 0:
        other = rbe.FP64 if prec == rbe.FP32C else rbe.FP32C
        oname = "fp64" if other == rbe.FP64 else "fp32c"
        ost, _ = batched(other, max(1, repeats // 2 + 1), False)
        forms[f"batched_{oname}"] = ost
        v32_loop, _ = loop_rate(rbe.FP32C, max(2, Kc // 2))
        forms["loop_fp64"] = {"particle_steps_per_s": v64_loop}
        forms["loop_fp32c"] = {"particle_steps_per_s": v32_loop}
        log(f"replica256: batched {oname} {ost['median_ms']:.3f} ms/step; loops {v64_loop:.3e} / {v32_loop:.3e}")
    nq = int(np.count_nonzero(cat["q"]))
    P = reps[0][0]["P"]
    roof = None
    if "batch" in kernels:
        work = pair_flops(counts) + (FLOPS_RHO_IK + FLOPS_GATHER_IK) * nq * P
        avg_s = kernels["batch"]["avg_us"] * 1e-6
        peak = PEAK_FP64_TFLOPS if prec == rbe.FP64 else PEAK_FP32_TFLOPS
        ach = work / avg_s / 1e12
        roof = dict(kernel="batch", bound="alu", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=measured_traffic("replica256", "batch", [edge, xsplit], prec_name), work_per_launch=work)
    eps = None
    if with_eps and not a.no_eps:
        eps = eps_batch(rbe, reps, cat, off, edge, xsplit, sizes)
        log(f"replica256: force errors {eps}")
    out = {
        "value": stats["particle_steps_per_s"],
        "ms_per_step": stats["median_ms"],
        "dtype": "f64" if prec == rbe.FP64 else "f32+f64",
        "config": {"workload": "replica256", "replicas": len(sizes), "n": ntot, "n_charged": nq,
                   "n_min": min(sizes), "n_max": max(sizes), "density": 0.5, "alpha": reps[0][0]["alpha"],
                   "r_coul": reps[0][0]["r_coul"], "r_lj": reps[0][0]["r_lj"], "P": P, "form": "batched " + prec_name,
                   "cell_edge": edge, "xsplit": xsplit, "tuned": tuned, "parallelism": "single GPU"},
        "timing": {k: v for k, v in stats.items() if k != "particle_steps_per_s"},
        "forms": {k: {kk: vv for kk, vv in v.items() if kk in ("particle_steps_per_s", "median_ms", "min_ms",
                                                                 "max_ms", "repeats")} for k, v in forms.items()},
        "kernels": kernels,
        "counts_per_eval": dict(zip(("coul_pairs", "lj_pairs", "candidates", "shell_members"), counts)),
        "roofline": roof,
        "epsilon": eps,
        "gen_s": round(t_gen, 2),
    }
    b = forms.get("batched_fp32c", {}).get("particle_steps_per_s")
    if b and "batched_fp64" in forms:
        out["batched_fp32c_over_batched_fp64"] = b / forms["batched_fp64"]["particle_steps_per_s"]
        out["batched_fp32c_over_loop_fp64"] = b / forms["loop_fp64"]["particle_steps_per_s"]
    if with_cpu and not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(reps)
    return out


def eps_batch(rbe, reps, cat, off, edge, xsplit, sizes, ev=3):
    """Every row and term of the smallest, a middle and the largest replica,
    batched FP32C and FP64, against the oracle (each replica draws its own
    mode sample from its stream seed)."""
    import numpy as np
    import torch

    import oracle
    from paper_2609_02694_amd import tune

    order = np.argsort(sizes)
    pick = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    refs = {}
    for r in pick:
        p, s = reps[r]
        m, w = oracle.sample_k(p["stream_seed"], ev, p["L"], p["alpha"], p["P"])
        refs[r] = oracle.total_force(s["x"], s["y"], s["z"], s["q"], s["id"], oracle.sys_from_preset(p), m, w,
                                     seed=p["seed"], ev=ev)
    out = {"replicas": [int(reps[r][0]["n"]) for r in pick]}
    for prec, name in ((rbe.FP32C, "batched_fp32c"), (rbe.FP64, "batched_fp64")):
        e = {}
        for t, mask in zip(TERM_NAMES + ("total",), (rbe.TERM_LJ, rbe.TERM_COUL_REAL, rbe.TERM_FOURIER,
                                                      rbe.TERM_ALL)):
            ctx = rbe.Context.batch(tune.batch_params(reps, edge, prec, xsplit, terms=mask), off)
            st = rbe.Particles.from_numpy(cat)
            ctx.forces(st, None, None, ev)
            torch.cuda.synchronize()
            ctx.sync_check()
            F = np.stack([st.fx.cpu().numpy(), st.fy.cpu().numpy(), st.fz.cpu().numpy()], axis=1)
            ctx.close()
            key = {"total": "F", "coul_real": "coul"}.get(t, t)
            num = sum(float(np.linalg.norm(F[off[r]:off[r + 1]] - refs[r][key]) ** 2) for r in pick)
            den = sum(float(np.linalg.norm(refs[r][key]) ** 2) for r in pick)
            e[t] = (num / den) ** 0.5
        out[name] = e
    return out


def cpu_baseline_batch(reps, budget_s=15.0):
    """The FP64 CPU oracle on one velocity-Verlet step of replicas taken in order until about budget_s."""
    import oracle

    done = 0
    t0 = time.perf_counter()
    k = 0
    for p, s in reps:
        q = dict(p, seed=p["stream_seed"])
        oracle_vv_step(q, s)
        done += p["n"]
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one velocity-Verlet step of the first {k} replicas ({done} particles)",
            "seconds": round(dt, 2)}


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the path runs on one GPU only; --gpus {a.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2609_02694_amd as rbe

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.calibrate_copy:
        return calibrate_copy(a.calibrate_copy)
    if a.calibrate_valu:
        return calibrate_valu(rbe)
    rbe.load()
    t_start = time.time()
    common = {"metric": METRIC, "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
              "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "data": "synthetic"}
    if a.workload == "headline":
        head = bench_single(a, rbe, "subdomain64m", "fp32c", a.repeats)
        batch = bench_batch(a, rbe, a.repeats)
        out = dict(common)
        out.update({k: head[k] for k in ("value", "ms_per_step", "dtype", "config")})
        out.update({k: v for k, v in head.items() if k not in ("value", "ms_per_step", "dtype", "config")})
        out["batched"] = batch
    elif a.workload == "replica256":
        out = dict(common)
        out.update(bench_batch(a, rbe, a.repeats))
    else:
        prec_name = a.prec or ("fp64" if a.workload in ("plain3k", "electrolyte1m", "ljelectrolyte") else "fp32c")
        out = dict(common)
        out.update(bench_single(a, rbe, a.workload, prec_name, a.repeats))
    out["bench_wall_s"] = round(time.time() - t_start, 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
