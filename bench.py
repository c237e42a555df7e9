"""Throughput of the RBE nonbonded force + velocity-Verlet step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--prec fp64|fp32c]

A step is one pass of the whole hot path over the system: half-kick + drift
+ wrap, cell binning and reorder, mode sample, near field (with the core-shell
random batch list where the workload has one), structure factors, Fourier
gather and the second half-kick. Inputs are synthetic (seeded generator) and
resident in HBM before the timed region. Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s RBE nonbonded force, FP32-comp & batched vs FP64, ≤1e-5 err"

# MI355X published peaks
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Algorithmic work per unit (FMA = 2 flops; a special function counts 1):
#   near field: per Coulomb pair term 27 flops, per LJ pair term 22 flops,
#               per ranked shell member 20 ops
#   structure factor: 13 flops per (charged particle, mode)
#   gather: 18 flops per (charged particle, mode)
FLOPS_COUL_PAIR = 27
FLOPS_LJ_PAIR = 22
OPS_SHELL_MEMBER = 20
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


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="electrolyte1m",
                    choices=["plain3k", "electrolyte1m", "ions8m", "subdomain64m", "replica256",
                             "ljelectrolyte"])
    ap.add_argument("--compare-steps", type=int, default=100,
                    help="steps of each comparison form (the other precision; replica256: FP64 and FP32C "
                         "per-replica loops and the other-precision batch); 0 skips them")
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
    ap.add_argument("--no-timing", action="store_true", help="skip the per-kernel HIP event timing")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (scale of the HBM byte counters)")
    return ap.parse_args()


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


def main():
    a = parse()
    if a.gpus != 1:
        print(f"bench.py: the path runs on one GPU only; --gpus {a.gpus} is not supported "
              "(sharding across GPUs is not implemented)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import gen
    import paper_2609_02694_amd as rbe

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if a.calibrate_copy:
        return calibrate_copy(a.calibrate_copy)
    rbe.load()
    if a.workload == "replica256":
        return bench_batch(a)
    p = gen.preset(a.workload, n=a.n)
    if a.rbl_shell:
        if a.rbl_shell == "charged" and not p.get("r_core", 0.0) > 0.0:
            print(f"--rbl-shell charged needs a workload with the random batch list ({a.workload} has none)",
                  file=sys.stderr)
            sys.exit(2)
        p["rbl_shell"] = 1 if a.rbl_shell == "charged" else 0
    prec_name = a.prec or ("fp64" if a.workload in ("plain3k", "electrolyte1m", "ljelectrolyte") else "fp32c")
    prec = rbe.FP64 if prec_name == "fp64" else rbe.FP32C
    h = a.edge or DEFAULT_NCELL_H.get(a.workload, 3.0)
    nc = max(1, int(p["L"] // h))
    nx = nc * (a.xsplit or DEFAULT_XSPLIT.get(a.workload, 1))
    t0 = time.time()
    s = gen.make_system(p)
    t_gen = time.time() - t0
    n = p["n"]
    tuned = None
    if a.tune:
        from paper_2609_02694_amd import tune
        t1 = time.time()
        (nx, nc, _), hit = tune.tune_grid_cached(p, s, prec, a.tune_cache, steps=10)
        tuned = dict(cache_hit=hit, seconds=round(time.time() - t1, 1))
    params = rbe.params_from_preset(p, prec=prec, ncell=(nx, nc, nc))
    ctx = rbe.Context(params, n)
    st = rbe.Particles.from_numpy(s)
    if p.get("nvt_tau", 0.0) > 0:
        st.nh = torch.zeros(2, dtype=torch.float64, device="cuda")  # Nose-Hoover {xi, eta}
    stream = torch.cuda.current_stream()

    # algorithmic counts of one force evaluation (counting pass, untimed)
    ctx.set_counting(True)
    ctx.forces(st, None, None, 0)
    cnt = ctx.counters()
    ctx.set_counting(False)
    nq = int(np.count_nonzero(s["q"]))
    ctx.forces(st, None, None, 0)  # initial force, eval 0
    ctx.sync_check()

    K, W = a.steps, a.warmup
    if W > 0:
        ctx.step(st, W, 1)
    torch.cuda.synchronize()
    ctx.sync_check()
    if not a.no_timing:
        ctx.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(st, K, 1 + W)
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    kt = ctx.timing() if not a.no_timing else {}
    ctx.set_timing(False)
    ctx.sync_check()
    wall_s = w1 - w0
    ev_ms = ev0.elapsed_time(ev1)
    value = n * K / wall_s

    kernels = {k: {"total_ms": round(v[0], 4), "launches": v[1], "avg_us": round(1000 * v[0] / v[1], 3)}
               for k, v in kt.items() if v[1] > 0}
    roof, roofs = roofline(kernels, cnt, nq, p, prec, K, workload=a.workload, grid=[nx, nc, nc])

    # the other precision form on the same system and grid (untimed in `value`)
    forms = {prec_name: value}
    if a.compare_steps > 0:
        other = rbe.FP32C if prec == rbe.FP64 else rbe.FP64
        oname = "fp32c" if other == rbe.FP32C else "fp64"
        octx = rbe.Context(rbe.params_from_preset(p, prec=other, ncell=(nx, nc, nc)), n)
        ost = rbe.Particles.from_numpy(s)
        if p.get("nvt_tau", 0.0) > 0:
            ost.nh = torch.zeros(2, dtype=torch.float64, device="cuda")
        octx.forces(ost, None, None, 0)
        octx.step(ost, 3, 1)
        if not a.no_timing:
            octx.set_timing(True)  # the same per-kernel events as the timed form
        torch.cuda.synchronize()
        t = time.perf_counter()
        octx.step(ost, a.compare_steps, 4)
        torch.cuda.synchronize()
        forms[oname] = n * a.compare_steps / (time.perf_counter() - t)
        octx.set_timing(False)
        octx.sync_check()
        octx.close()

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * wall_s / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == rbe.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "n": n, "n_charged": nq, "L": round(p["L"], 4), "alpha": p["alpha"],
                   "r_coul": p["r_coul"], "r_lj": p["r_lj"], "r_core": p["r_core"], "p_shell": p["p_shell"],
                   "P": p["P"], "dt": p["dt"], "form": prec_name, "ncell": [nx, nc, nc], "tuned": tuned,
                   "ensemble": "NVT" if p.get("nvt_tau", 0.0) > 0 else "NVE",
                   "rbl_shell": "charged" if p.get("rbl_shell", 0) else "all",
                   "parallelism": "single GPU"},
        "event_ms_per_step": ev_ms / K,
        "kernels": kernels,
        "counts_per_eval": {k: dict(zip(("coul_pairs", "lj_pairs", "candidates", "shell_members"), v))
                            for k, v in cnt.items()},
        "roofline": roof,
        "rooflines": roofs,
        "forms_particle_steps_per_s": forms,
        "gen_s": round(t_gen, 2),
    }
    ctx.close()
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, s)
    print(json.dumps(out), flush=True)


def bench_batch(a):
    """256 replicas of uneven size advanced together by the batched form."""
    import numpy as np
    import torch

    import gen
    import paper_2609_02694_amd as rbe
    from paper_2609_02694_amd import tune

    prec_name = a.prec or "fp32c"
    prec = rbe.FP64 if prec_name == "fp64" else rbe.FP32C
    t0 = time.time()
    sizes = gen.replica_sizes(256)
    reps, cat, off = gen.replica_batch(sizes)
    t_gen = time.time() - t0
    ntot = int(off[-1])
    edge = a.edge or DEFAULT_NCELL_H["replica"]
    xsplit = a.xsplit or DEFAULT_XSPLIT["replica"]
    tuned = None
    if a.tune:
        t1 = time.time()
        (edge, xsplit), hit = tune.tune_batch_cached(reps, cat, off, prec, a.tune_cache, steps=5)
        tuned = dict(cache_hit=hit, seconds=round(time.time() - t1, 1))
    ctx = rbe.Context.batch(tune.batch_params(reps, edge, prec, xsplit), off)
    st = rbe.Particles.from_numpy(cat)
    stream = torch.cuda.current_stream()
    ctx.forces(st, None, None, 0)
    K, W = a.steps, a.warmup
    if W > 0:
        ctx.step(st, W, 1)
    torch.cuda.synchronize()
    ctx.sync_check()
    if not a.no_timing:
        ctx.set_timing(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record(stream)
    ctx.step(st, K, 1 + W)
    ev1.record(stream)
    torch.cuda.synchronize()
    w1 = time.perf_counter()
    kt = ctx.timing() if not a.no_timing else {}
    ctx.set_timing(False)
    ctx.sync_check()
    ctx.close()
    wall_s = w1 - w0
    value = ntot * K / wall_s
    kernels = {k: {"total_ms": round(v[0], 4), "launches": v[1], "avg_us": round(1000 * v[0] / v[1], 3)}
               for k, v in kt.items() if v[1] > 0}

    # comparison forms (same replicas, same grids): per-replica loops of
    # single-system contexts in FP64 and FP32C, and the batched form in FP64
    def loop_rate(pr, steps):
        """particle-steps/s of a loop of single-system contexts (0 steps: only the
        pair counts of one evaluation, FP64 contexts)."""
        ctxs, sts = [], []
        for (p, s) in reps:
            n = max(1, int(p["L"] // edge))
            ctxs.append(rbe.Context(rbe.params_from_preset(p, prec=pr, ncell=(xsplit * n, n, n), seed=p["stream_seed"]),
                                    p["n"]))
            sts.append(rbe.Particles.from_numpy(s))
        rate = None
        if steps > 0:
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

    Kc = max(2, a.compare_steps // 5) if a.compare_steps > 0 else 0
    v64_loop, counts = loop_rate(rbe.FP64, Kc)
    forms = {f"batched_{prec_name}": value}
    if a.compare_steps > 0:
        v32_loop, _ = loop_rate(rbe.FP32C, Kc)
        other = rbe.FP64 if prec == rbe.FP32C else rbe.FP32C
        ms_other = tune.time_batch(reps, cat, off, edge, other, steps=a.compare_steps, xsplit=xsplit)
        forms[f"batched_{'fp64' if other == rbe.FP64 else 'fp32c'}"] = ntot / (ms_other * 1e-3)
        forms["loop_fp64"] = v64_loop
        forms["loop_fp32c"] = v32_loop
    nq = int(np.count_nonzero(cat["q"]))
    P = reps[0][0]["P"]
    roof = None
    if "batch" in kernels:
        work = FLOPS_COUL_PAIR * counts[0] + FLOPS_LJ_PAIR * counts[1] + (FLOPS_RHO_IK + FLOPS_GATHER_IK) * nq * P
        avg_s = kernels["batch"]["avg_us"] * 1e-6
        peak = PEAK_FP64_TFLOPS if prec == rbe.FP64 else PEAK_FP32_TFLOPS
        ach = work / avg_s / 1e12
        roof = dict(kernel="batch", bound="alu", achieved=ach, peak=peak, unit="TFLOP/s", frac=ach / peak,
                    traffic=measured_traffic("replica256", "batch", [edge, xsplit]), work_per_launch=work)
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": 1000.0 * wall_s / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == rbe.FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "replica256", "replicas": len(sizes), "n": ntot, "n_charged": nq,
                   "n_min": min(sizes), "n_max": max(sizes), "density": 0.5, "alpha": reps[0][0]["alpha"],
                   "r_coul": reps[0][0]["r_coul"], "r_lj": reps[0][0]["r_lj"], "P": P, "form": "batched " + prec_name,
                   "cell_edge": edge, "xsplit": xsplit, "tuned": tuned, "parallelism": "single GPU"},
        "event_ms_per_step": ev0.elapsed_time(ev1) / K,
        "kernels": kernels,
        "forms_particle_steps_per_s": forms,
        "counts_per_eval": dict(zip(("coul_pairs", "lj_pairs", "candidates", "shell_members"), counts)),
        "roofline": roof,
        "gen_s": round(t_gen, 2),
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(reps)
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(reps, budget_s=15.0):
    """The FP64 CPU oracle on one velocity-Verlet step of replicas taken in order until about budget_s."""
    import numpy as np

    import oracle

    done = 0
    t0 = time.perf_counter()
    k = 0
    for p, s in reps:
        osys = oracle.sys_from_preset(p)
        m, w = oracle.sample_k(p["stream_seed"], 1, p["L"], p["alpha"], p["P"])
        r = np.stack([s["x"], s["y"], s["z"]], axis=1)
        v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)
        v = oracle.kick(np.zeros_like(r), v, p["dt"] / 2)
        r = oracle.drift_wrap(r, v, p["dt"], p["L"])
        F = oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, m, w, ev=1, components=False)["F"]
        v = oracle.kick(F, v, p["dt"] / 2)
        done += p["n"]
        k += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return {"value": done / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one velocity-Verlet step of the first {k} replicas ({done} particles)",
            "seconds": round(dt, 2)}


# Fourier kernels, issue-slot model: per (charged particle, mode) two
# transcendentals (sin, cos of the phase; quarter rate, 4 lane slots each)
# plus 5 FP64 phase operations and 2 (structure factor) or 5 (gather) FMAs;
# against 256 CU x 64 lanes x 2.4 GHz = 39.3 T lane-slots/s.
PEAK_LANE_SLOTS_T = 256 * 64 * 2.4e9 / 1e12
SLOTS_RHO_IK = 2 * 4 + 5 + 2
SLOTS_GATHER_IK = 2 * 4 + 5 + 5


def kernel_roofline(name, kernels, cnt, nq, p, prec):
    """Roofline entry of one timed kernel kind (None if no model applies)."""
    if name not in kernels:
        return None
    avg_s = kernels[name]["avg_us"] * 1e-6
    peak_alu = PEAK_FP64_TFLOPS if prec == 0 else PEAK_FP32_TFLOPS
    n, P = p["n"], p["P"]
    if name.startswith("pair") and cnt and name in cnt:
        c = cnt[name]
        work = FLOPS_COUL_PAIR * c[0] + FLOPS_LJ_PAIR * c[1] + OPS_SHELL_MEMBER * c[3]
        ach = work / avg_s / 1e12
        return dict(kernel=name, bound="alu", achieved=ach, peak=peak_alu, unit="TFLOP/s", frac=ach / peak_alu,
                    work_per_launch=work)
    if name in ("rho_partial", "gather"):
        per = SLOTS_RHO_IK if name == "rho_partial" else SLOTS_GATHER_IK
        work = per * nq * P
        ach = work / avg_s / 1e12
        return dict(kernel=name, bound="alu", achieved=ach, peak=PEAK_LANE_SLOTS_T, unit="Tslot/s",
                    frac=ach / PEAK_LANE_SLOTS_T, work_per_launch=work)
    per_bytes = {"kick_drift": BYTES_KICK_DRIFT, "kick": BYTES_KICK}.get(name)
    if per_bytes is None:
        return None
    ach = per_bytes * n / avg_s / 1e9
    return dict(kernel=name, bound="hbm", achieved=ach, peak=PEAK_HBM_GBS, unit="GB/s", frac=ach / PEAK_HBM_GBS,
                work_per_launch=per_bytes * n)


def measured_traffic(workload, name, grid=None):
    """HBM bytes per launch of a kernel kind from the committed rocprofv3 counter
    runs (profiles/traffic.json), or None when the kernel sources or the cell
    grid differ from the counted run."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path)).get(workload)
    if not d or name not in d.get("kinds", {}):
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


def roofline(kernels, cnt, nq, p, prec, K, workload=None, grid=None):
    """Roofline figure of the dominant kernel (largest summed time), and of every kind with a model."""
    if not kernels:
        return None, {}
    every = {k: kernel_roofline(k, kernels, cnt, nq, p, prec) for k in kernels}
    every = {k: v for k, v in every.items() if v}
    name = max(kernels, key=lambda k: kernels[k]["total_ms"])
    dom = every.get(name) or dict(kernel=name, bound="alu", achieved=None, peak=None, unit=None, frac=None)
    dom = dict(dom)
    dom["traffic"] = measured_traffic(workload, name, grid) if workload else None
    # counted HBM bytes per launch over the live average duration, against the
    # HBM peak (shown for every kind, whatever bounds it)
    for k, r in [(name, dom)] + list(every.items()):
        t = dom["traffic"] if k == name else (measured_traffic(workload, k, grid) if workload else None)
        if t and kernels[k]["avg_us"] > 0:
            r["hbm_gbps"] = t / (kernels[k]["avg_us"] * 1e-6) / 1e9
            r["hbm_frac"] = r["hbm_gbps"] / PEAK_HBM_GBS
    return dom, every


def cpu_baseline(p, s):
    """The FP64 CPU oracle on one velocity-Verlet step of the same system."""
    import numpy as np

    import oracle

    osys = oracle.sys_from_preset(p)
    t0 = time.perf_counter()
    m, w = oracle.sample_k(p["seed"], 1, p["L"], p["alpha"], p["P"])
    r = np.stack([s["x"], s["y"], s["z"]], axis=1)
    v = np.stack([s["vx"], s["vy"], s["vz"]], axis=1)
    F0 = np.zeros_like(r)
    v = oracle.kick(F0, v, p["dt"] / 2)
    r = oracle.drift_wrap(r, v, p["dt"], p["L"])
    F = oracle.total_force(r[:, 0], r[:, 1], r[:, 2], s["q"], s["id"], osys, m, w, seed=p["seed"], ev=1,
                             components=False)["F"]
    v = oracle.kick(F, v, p["dt"] / 2)
    dt = time.perf_counter() - t0
    cpu = None
    try:
        with open("/proc/cpuinfo") as f:
            cpu = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": p["n"] / dt, "unit": "particle-steps/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"one velocity-Verlet step (one force evaluation) of the full {p['n']}-particle system",
            "seconds": round(dt, 2), "cpu_model": cpu}


if __name__ == "__main__":
    main()
