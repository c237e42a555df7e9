"""Radial distribution functions of the implicit-solvent LJ electrolyte
(Sec. 3.1, with the force parameters of the paper's parameter table: r_s = 8,
r_c = 4, p = 30, P = 200, dt = 0.001, Nose-Hoover at kT = 1), simulated with
RBE + random batch list and with plain Ewald, as in the paper's accuracy
check (Sec. 3.2), at a reduced particle count and the same number density.

Both runs go through the library: `rbe_step` with the sampled modes of Eq. 9
and the core-shell list of Eq. 10-11, and `rbe_step` with the Ewald lattice
table fixed by `rbe_set_modes` (every mode with exp(-k^2/4 alpha) above
--ewald-tail, r_c = 0: every pair inside r_s summed). They start from the same
seeded configuration, equilibrate, then sample g(r) of cation-cation and
cation-anion pairs every --every steps. The statistical error of each curve is
the spread of its block averages.

    python3 rdf_compare.py [--n 4000] [--equil 5000] [--steps 20000] [--every 100]

prints one JSON line (and writes it to --out when given).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=4000)
    ap.add_argument("--equil", type=int, default=5000)
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--every", type=int, default=100)
    ap.add_argument("--blocks", type=int, default=5)
    ap.add_argument("--rmax", type=float, default=8.0)
    ap.add_argument("--dr", type=float, default=0.1)
    ap.add_argument("--ewald-tail", type=float, default=1e-7)
    ap.add_argument("--forms", default="ewald,rbe64,rbe32c",
                    help="comma list: ewald, rbe64, rbe32c, each optionally with :P<modes>, :rc<core radius> "
                         "and :dt<step> (e.g. rbe64:P1000, rbe64:rc0 (no batch list), rbe64:dt0.0005; a "
                         "smaller dt runs proportionally more steps)")
    ap.add_argument("--seeds", default="1006",
                    help="comma list of seeds: each form runs once per seed (independent initial state and "
                         "mode stream); the curves are averaged over seeds and their error is the spread "
                         "between seeds (with one seed, between block averages)")
    ap.add_argument("--ref", default=None, help="take the ewald curves from this earlier output instead of running it")
    ap.add_argument("--out", default=None)
    return ap.parse_args()


def log(msg):
    print(f"rdf: {msg}", file=sys.stderr, flush=True)


def histograms(x, y, z, q, L, edges):
    """Pair-distance histograms (cation-cation, cation-anion) of one snapshot,
    minimum image (rmax < L/2)."""
    import torch
    r = torch.stack([x, y, z], dim=1)
    cat, an = r[q > 0], r[q < 0]
    out = []
    for a, b, same in ((cat, cat, True), (cat, an, False)):
        d = a[:, None, :] - b[None, :, :]
        d = d - L * torch.round(d / L)
        dist = torch.sqrt((d * d).sum(dim=2))
        if same:
            iu = torch.triu_indices(len(a), len(a), offset=1, device=dist.device)
            dist = dist[iu[0], iu[1]]
        else:
            dist = dist.reshape(-1)
        out.append(torch.histc(dist, bins=len(edges) - 1, min=edges[0], max=edges[-1]).double())
    return out, len(cat), len(an)


def parse_form(spec, p):
    """'rbe64:P1000:rc0:dt0.0005' -> (kind, preset with the overrides, step scale)."""
    parts = spec.split(":")
    kind, pr, scale = parts[0], dict(p), 1
    if kind not in ("ewald", "rbe64", "rbe32c"):
        raise SystemExit(f"unknown form {spec}")
    for o in parts[1:]:
        if o.startswith("P"):
            pr["P"] = int(o[1:])
        elif o.startswith("rc"):
            pr["r_core"] = float(o[2:])
            if pr["r_core"] == 0.0:
                pr["p_shell"] = 0
        elif o.startswith("dt"):
            pr["dt"] = float(o[2:])
            scale = max(1, int(round(p["dt"] / pr["dt"])))
        else:
            raise SystemExit(f"unknown option {o} in {spec}")
    return kind, pr, scale


def run(spec, p, s, a, edges):
    import numpy as np
    import torch
    import paper_2609_02694_amd as rbe
    form, pr, scale = parse_form(spec, p)
    prec = rbe.FP32C if form == "rbe32c" else rbe.FP64
    if form == "ewald":
        pr.update(r_core=0.0, p_shell=0)
    params = rbe.params_from_preset(pr, prec=prec)
    info = {}
    if form == "ewald":
        kmax = math.sqrt(4.0 * p["alpha"] * math.log(1.0 / a.ewald_tail))
        m, w = rbe.lattice_modes(params, kmax)
        params.P = m.shape[1]
        info = dict(k_max=kmax, modes=int(params.P))
    ctx = rbe.Context(params, p["n"])
    st = rbe.Particles.from_numpy(s)
    st.nh = torch.zeros(2, dtype=torch.float64, device="cuda")
    if form == "ewald":
        ctx.set_modes(torch.as_tensor(m.ravel()).cuda(), torch.as_tensor(w).cuda())
    equil, steps, every = a.equil * scale, a.steps * scale, a.every * scale
    form = spec
    log(f"{form}: n={p['n']} L={p['L']:.3f} P={params.P} r_core={pr['r_core']} dt={pr['dt']} {info}")
    ctx.forces(st, None, None, 0)
    ev = 1
    t0 = time.perf_counter()
    done = 0
    while done < equil:
        k = min(1000 * scale, equil - done)
        ctx.step(st, k, ev)
        ev += k
        done += k
        torch.cuda.synchronize()
        log(f"{form}: equilibration {done}/{equil} steps")
    nbin = len(edges) - 1
    per_block = max(1, (steps // every) // a.blocks)
    blocks = []
    acc = [torch.zeros(nbin, dtype=torch.float64, device="cuda") for _ in range(2)]
    nsnap = 0
    temps = []
    for snap in range(steps // every):
        ctx.step(st, every, ev)
        ev += every
        h, ncat, nan = histograms(st.x, st.y, st.z, st.q, p["L"], edges)
        for c in range(2):
            acc[c] += h[c]
        nsnap += 1
        v2 = (st.vx * st.vx + st.vy * st.vy + st.vz * st.vz).sum()
        temps.append(float(v2) / (3 * p["n"] - 3))
        if nsnap == per_block:
            blocks.append([c.cpu().numpy() / nsnap for c in acc])
            acc = [torch.zeros(nbin, dtype=torch.float64, device="cuda") for _ in range(2)]
            nsnap = 0
            log(f"{form}: block {len(blocks)} done ({snap + 1} snapshots, kT {np.mean(temps[-per_block:]):.3f})")
    torch.cuda.synchronize()
    ctx.sync_check()
    secs = time.perf_counter() - t0
    ctx.close()
    # normalisation: ideal-gas pair counts in each shell
    V = p["L"] ** 3
    shell = 4.0 / 3.0 * math.pi * (edges[1:] ** 3 - edges[:-1] ** 3)
    ideal = [ncat * (ncat - 1) / 2 * shell / V, ncat * nan * shell / V]
    g = [np.array([b[c] / ideal[c] for b in blocks]) for c in range(2)]
    return dict(form=form, P=int(params.P), dt=pr["dt"], seconds=secs, steps=equil + steps,
                kT_mean=float(np.mean(temps)),
                g_cc=g[0].mean(axis=0), g_ca=g[1].mean(axis=0),
                se_cc=g[0].std(axis=0, ddof=1) / math.sqrt(len(blocks)),
                se_ca=g[1].std(axis=0, ddof=1) / math.sqrt(len(blocks)), **info)


def main():
    import numpy as np
    import torch
    import gen
    a = parse()
    if not torch.cuda.is_available():
        raise SystemExit("rdf_compare.py needs a GPU")
    seeds = [int(x) for x in a.seeds.split(",") if x]
    p = gen.preset("ljelectrolyte", n=a.n)
    if a.rmax >= p["L"] / 2:
        raise SystemExit("rmax must stay below L/2")
    edges = np.arange(0.0, a.rmax + 0.5 * a.dr, a.dr)
    res = {}
    if a.ref:
        ref = json.loads(open(a.ref).read().strip().splitlines()[-1])
        e = ref["ewald"]
        res["ewald"] = {k: (np.array(v) if isinstance(v, list) else v) for k, v in e.items()}
    for f in a.forms.split(","):
        if not f or f in res:
            continue
        runs = []
        for sd in seeds:
            ps = dict(p, seed=sd)
            runs.append(run(f, ps, gen.make_system(ps), a, edges))
        if len(runs) == 1:
            res[f] = runs[0]
            continue
        agg = dict(runs[0], seeds=seeds, seconds=sum(x["seconds"] for x in runs),
                   kT_mean=float(np.mean([x["kT_mean"] for x in runs])))
        for key in ("cc", "ca"):
            gs = np.array([x["g_" + key] for x in runs])
            agg["g_" + key] = gs.mean(axis=0)
            agg["se_" + key] = gs.std(axis=0, ddof=1) / math.sqrt(len(runs))
            agg["g_" + key + "_per_seed"] = gs
        res[f] = agg
    r = 0.5 * (edges[1:] + edges[:-1])
    out = dict(system=dict(preset="ljelectrolyte", n=p["n"], L=p["L"], density=p["n"] / p["L"] ** 3,
                           alpha=p["alpha"], r_s=p["r_coul"], r_lj=p["r_lj"], r_c=p["r_core"], p=p["p_shell"],
                           P=p["P"], dt=p["dt"], kT=p["nvt_kT"], tau=p["nvt_tau"]),
               protocol=dict(equil=a.equil, steps=a.steps, every=a.every, blocks=a.blocks, dr=a.dr, seeds=seeds),
               r=r.tolist())
    for f, v in res.items():
        out[f] = {k: (val.tolist() if hasattr(val, "tolist") else val) for k, val in v.items()}
    if "ewald" in res:
        e = res["ewald"]
        # compare where the curves carry weight (g > 0.05 in the reference)
        for f in res:
            if f == "ewald":
                continue
            cmp = {}
            for key in ("cc", "ca"):
                ge, gf = e["g_" + key], res[f]["g_" + key]
                se = np.sqrt(e["se_" + key] ** 2 + res[f]["se_" + key] ** 2)
                mask = ge > 0.05
                d = np.abs(gf - ge)[mask]
                z = (np.abs(gf - ge) / np.where(se > 0, se, np.inf))[mask]
                cmp[key] = dict(max_abs_diff=float(d.max()), r_at_max=float(r[mask][np.argmax(d)]),
                                rms_diff=float(np.sqrt((d ** 2).mean())), max_z=float(z.max()),
                                frac_bins_within_2se=float((z <= 2).mean()), peak_ref=float(ge.max()),
                                r_peak_ref=float(r[np.argmax(ge)]), peak=float(gf.max()),
                                r_peak=float(r[np.argmax(gf)]))
            out["vs_ewald_" + f] = cmp
            log(f"{f} vs ewald: {cmp}")
    line = json.dumps(out)
    print(line, flush=True)
    if a.out:
        with open(a.out, "w") as fh:
            fh.write(line + "\n")


if __name__ == "__main__":
    main()
