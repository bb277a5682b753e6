"""Benchmark: particle-steps per second of the Ito-KMC step on one MI355X.

A step is one pass of the whole path (push with fused NGP binning, photon transport,
counting sort by cell, per-cell KMC, coupling, and in the self-consistent workload the
charge deposit and field solve) over the resident particles.  Inputs are seeded and
synthetic and resident in HBM before the timed region starts.

Prints one JSON line.  `roofline` reports the dominant kernel's algorithmic bytes per
launch over its average launch time (HIP events recorded by the library on its own
stream during the timed steps) against the 8 TB/s HBM peak.  `cpu_baseline` times
the FP64 oracle on a bounded sample of the same workload on one host core.
"""
import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Single-kernel phases timed with HIP events (library profiling mode), the kernel each
# one is, and its algorithmic HBM bytes per unit (S = 4 in single, 8 in double precision):
#   push / field_push (per live particle): read cell 4 + offsets 3S + id 8 + weight 4,
#                      write cell 4 + offsets 3S + rank 4; field_push also reads the
#                      particle's mobility (S) that the deposit kept
#   deposit (per particle): read cell 4 + offsets 3S + id 8 + weight 4, write the
#                      particle's mobility S
#   scatter (per particle): read cell 4 + rank 4 + offsets 3S + weight 4 + id 8, write
#                      cell 4 + offsets 3S + weight 4 + id 8
#   couple (per particle gathered by the wavefront-per-cell coupling kernel: cells that
#                      merge or hold many particles): read and write cell, offsets,
#                      weight and id; without merging (n_ppc = 0) the kernel only removes
#                      weight, reading each gathered particle's weight and id (12 B)
#   smooth_fine (per finest-level cell and launch of one colour, split red-black order):
#                      read u and eps of the other colour's cells, f and eps of the
#                      colour's cells, write u of the colour's cells: 2.5 S
#   ions (per cell and move, mobile ions only; the three passes together): clear the
#                      next counts (write 8), read the counts (8), copy back (read 8,
#                      write 8): 32; the field and the atomics of ion-holding cells are
#                      not counted
KERNELS = {"push": "k_push_uniform", "field_push": "k_push_field", "deposit": "k_field_deposit_lds",
           "scatter": "k_scatter", "couple": "k_couple", "smooth_fine": "k_smooth_seg<fine>",
           "ions": "k_ion_move"}


def bytes_per_unit(phase, S):
    return {"push": 24 + 6 * S, "field_push": 24 + 7 * S, "deposit": 16 + 4 * S,
            "scatter": 36 + 6 * S, "couple": 32 + 6 * S, "smooth_fine": 5 * S / 2,
            "ions": 32}[phase]


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=20)
    p.add_argument("--workload", default="streamer_256")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=12.0)
    # batched ensemble (--workload ensemble_256) and served (--workload served) forms
    p.add_argument("--realizations", type=int, default=256)
    p.add_argument("--rate", type=float, default=200.0)
    p.add_argument("--duration", type=float, default=60.0)
    p.add_argument("--poisson-frac", type=float, default=0.004)
    p.add_argument("--budget-gb", type=float, default=200.0)
    p.add_argument("--drain", type=float, default=60.0)
    p.add_argument("--poisson-workers", type=int, default=8)
    p.add_argument("--reactor-frac", type=float, default=0.0,
                   help="served workload: share of zero-dimensional reactor requests")
    p.add_argument("--copy-calibration", action="store_true",
                   help="first copy 1 GiB device to device (a known-size kernel for "
                        "scaling hardware traffic counters)")
    p.add_argument("--no-plain", action="store_true")
    p.add_argument("--no-scale-window", action="store_true",
                   help="skip the second timed window near the particle cap")
    p.add_argument("--scale-steps", type=int, default=8)
    p.add_argument("--cpu-workers", type=int, default=16,
                   help="oracle processes of the multi-core host baseline (0: skip)")
    return p.parse_args()


def traffic_from_profile(kernel_label, workload, key="hbm_bytes_per_launch"):
    """Measured HBM bytes per launch (or another recorded quantity, e.g.
    valu_busy_pct) of a kernel on a workload from a committed counter summary
    (profiles/*_traffic.md, lines `key: value`), or None when there is none or when a
    source file it names has changed since the counters were taken."""
    import glob
    import hashlib
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md"))):
        kv = {}
        for line in open(path):
            m = re.match(r"^- (\w+): (.+)$", line.strip())
            if m:
                kv[m.group(1)] = m.group(2).strip()
        if kv.get("kernel") != kernel_label or kv.get("workload") != workload or "sources" not in kv:
            continue
        h = hashlib.sha256()
        for rel in kv["sources"].split():
            src = os.path.join(ROOT, rel)
            if not os.path.exists(src):
                return None
            h.update(open(src, "rb").read())
        if h.hexdigest() != kv.get("source_sha256") or key not in kv:
            return None
        return float(kv[key]) if "." in kv[key] else int(kv[key])
    return None


def cpu_baseline(cfg, budget_s):
    """Oracle (plain FP64, single thread) on a bounded sample of the workload: the same
    grid and physics with fewer seed electrons, stepped until the time budget."""
    import oracle
    from paper_2307_01797_amd import workloads
    scale = 200_000
    if cfg.get("seed_kind") == "gaussian":
        o = oracle.Sim(cfg)
        n0 = min(cfg["seed_n0"], scale)
        o.seed_gaussian(n0, cfg["seed_centre"], cfg["seed_sigma"])
        sample = f"{n0} seed electrons (of {cfg['seed_n0']}) on the full grid"
    else:
        # the oracle's conjugate-gradient solve at 256^3 takes minutes per step; the
        # sample is the same gap, seed and physics on the 64^3 grid
        sub = workloads.preset("streamer_64") if cfg["grid"][0] > 64 else cfg
        o = oracle.Sim(sub)
        o.seed_neutral(sub["seed_peak"], sub["seed_centre"], sub["seed_sigma"])
        sample = f"same streamer workload on the {sub['grid'][0]}^3 grid"
    psteps = 0
    t0 = time.perf_counter()
    nsteps = 0
    while time.perf_counter() - t0 < budget_s and nsteps < 50:
        psteps += o.diagnostics()["n_particles"]
        o.step(cfg["dt"], 1)
        nsteps += 1
    el = time.perf_counter() - t0
    return {"value": psteps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}, {nsteps} steps, {psteps} particle-steps in {el:.1f} s"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


# One oracle process of the multi-core host baseline: the streamer sample of
# cpu_baseline with realization r, stepped for a time budget; prints particle-steps and
# seconds.
_CPU_WORKER = r"""
import sys, time
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2307_01797_amd import workloads
r, budget = int(sys.argv[2]), float(sys.argv[3])
cfg = workloads.preset("streamer_64", realization=r)
o = oracle.Sim(cfg)
o.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
ps, t0, k = 0, time.perf_counter(), 0
while time.perf_counter() - t0 < budget and k < 50:
    ps += o.diagnostics()["n_particles"]
    o.step(cfg["dt"], 1)
    k += 1
print(ps, time.perf_counter() - t0, k)
"""


def cpu_baseline_parallel(workers, budget_s):
    """The oracle as it stands on several host cores at once: one single-threaded
    process per core, each a different realization of the streamer sample of
    cpu_baseline, started as child processes; the aggregate particle-steps/s."""
    import subprocess
    procs = [subprocess.Popen([sys.executable, "-c", _CPU_WORKER, ROOT, str(r), str(budget_s)],
                              stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True)
             for r in range(workers)]
    rate, steps = 0.0, []
    for pr in procs:
        out, _ = pr.communicate()
        ps, el, k = out.split()
        rate += int(ps) / float(el)
        steps.append(int(k))
    return {"value": rate, "unit": "particle-steps/s", "cores": workers, "kind": "oracle",
            "sample": f"{workers} processes (one per core), each the streamer workload on the "
                      f"64^3 grid with its own realization, {min(steps)}-{max(steps)} steps in "
                      f"about {budget_s:.0f} s"}


def cpu_baseline_ensemble(cfgs, budget_s):
    """Oracle on a stratified sample of the batched realizations (one per grid edge,
    in turn), each advanced step by step until the time budget is spent."""
    import oracle
    by_edge = {}
    for c in cfgs:
        by_edge.setdefault(c["grid"][0], c)
    sims = []
    for c in by_edge.values():
        o = oracle.Sim(c)
        o.seed_gaussian(c["seed_n0"], c["seed_centre"], c["seed_sigma"])
        sims.append([o, c, 0])
    psteps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        progressed = False
        for s in sims:
            o, c, k = s
            if k >= c["steps"]:
                continue
            psteps += o.diagnostics()["n_particles"]
            o.step(c["dt"], 1)
            s[2] += 1
            progressed = True
        if not progressed:
            break
    el = time.perf_counter() - t0
    steps = [s[2] for s in sims]
    return {"value": psteps / el, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one realization per grid edge {sorted(by_edge)}, steps {steps}, "
                      f"{psteps} particle-steps in {el:.1f} s"}


BYTES_EXPLICIT_STEP = 48 + 60   # push with binning + scatter, per particle-step


def step_forms(ens, best, rounds=2, per=3):
    """Mean step time of the ensemble step as its kernel sequence and as the persistent
    fused kernel at each register budget (1, 2, 4 workgroups per CU), interleaved over
    rounds on the warm-up ensemble; the autotuned shapes are restored afterwards."""
    import torch
    forms = [0, 1, 2, 4]
    tot = dict.fromkeys(forms, 0.0)
    for k in forms:                    # capture each form's graphs outside the timing
        ens.set_tuning(fused_per_cu=k)
        ens.step(1)
    for _ in range(rounds):
        for k in forms:
            ens.set_tuning(fused_per_cu=k)
            ens.step(1)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ens.step(per)
            ens.poll()
            tot[k] += time.perf_counter() - t0
    ens.set_tuning(**best)
    names = {0: "sequence", 1: "fused_1", 2: "fused_2", 4: "fused_4"}
    return {names[k]: round(1e3 * tot[k] / (rounds * per), 4) for k in forms}


def bench_ensemble(args):
    """Batched form: every realization in one ensemble, stepped together to the end,
    against the plain form (each realization alone in a single context)."""
    import torch

    from paper_2307_01797_amd import serve, workloads
    cfgs = workloads.ensemble_realizations(args.realizations)
    ens = serve.ensemble_for(cfgs)
    # warm-up pass: admit everything, run a few steps, pick launch shapes, release
    for i, c in enumerate(cfgs):
        ens.admit(c, tag=i)
    ens.step(max(1, args.warmup))
    tune, tune_ms = ens.autotune(rounds=2)
    forms_ms = step_forms(ens, tune)
    ens.poll()
    for s in list(ens.ncell):
        ens.release(s)
    ens.step(1)
    torch.cuda.synchronize()
    rb = serve.run_batched(cfgs, ens=ens, steps_per_poll=4)
    value = rb["particle_steps"] / rb["seconds"]
    steps_run = [r["step"] for r in rb["results"]]
    out = {
        "metric": "particle-steps/s (batched ensemble: push+sort+KMC+coupling)",
        "value": value, "unit": "particle-steps/s", "n_gpus": 1,
        "steps": int(max(steps_run)), "warmup": args.warmup,
        "ms_per_step": rb["seconds"] * 1e3 / max(1, max(steps_run)),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"ensemble_{len(cfgs)}", "realizations": len(cfgs),
                   "edges": sorted({c["grid"][0] for c in cfgs}), "dx_m": 5e-6,
                   "steps_max": 500, "stop_particles": 1_000_000,
                   "capped": sum(1 for r in rb["results"] if r["state"] != 2),
                   "particle_steps": rb["particle_steps"], "seconds": rb["seconds"],
                   "tuning": tune, "autotune_step_ms": tune_ms, "step_forms_ms": forms_ms,
                   "arena_gb": ens.arena_bytes / 1e9},
        "step_bandwidth": {"bytes_per_particle_step": BYTES_EXPLICIT_STEP,
                           "achieved_gbs": BYTES_EXPLICIT_STEP * value / 1e9,
                           "frac": BYTES_EXPLICIT_STEP * value / 1e9 / HBM_PEAK_GBS},
    }
    if not args.no_plain:
        log(f"batched form done in {rb['seconds']:.2f} s; plain form next")
        rp = serve.run_plain(cfgs, log=log)
        same = sum(1 for a, b in zip(rb["results"], rp["results"])
                   if all(a[k] == b[k] for k in ("weight", "n_particles", "fires", "n_plus",
                                                 "n_minus", "particle_steps", "step")))
        out["plain_form"] = {"seconds": rp["seconds"],
                             "value": rp["particle_steps"] / rp["seconds"],
                             "identical_results": same, "of": len(cfgs)}
        out["speedup_vs_plain"] = rp["seconds"] / rb["seconds"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_ensemble(cfgs, args.cpu_seconds)
    print(json.dumps(out))


def bench_served(args):
    """Served form: Poisson arrivals, continuous batching, HBM-budget admission;
    p50/p99 time-to-result beside throughput, against first-come first-served
    single-context serving of the same request stream."""
    import torch

    from paper_2307_01797_amd import serve, workloads
    trace = workloads.request_trace(rate=args.rate, duration=args.duration,
                                    poisson_frac=args.poisson_frac, reactor_frac=args.reactor_frac)
    srv = serve.Server(budget_bytes=args.budget_gb * 1e9, poisson_workers=args.poisson_workers)
    # warm-up: a few requests through both lanes (graph capture, allocator)
    warm = [(0.0, -1 - i, c) for i, (_, _, c) in enumerate(trace[:8])]
    srv.run(warm)
    torch.cuda.synchronize()
    summary, recs = srv.run(trace, drain_limit_s=args.drain, log=log)
    out = {
        "metric": "served requests/s with p50/p99 time-to-result",
        "value": summary["throughput_req_s"], "unit": "requests/s", "n_gpus": 1,
        "steps": summary["ensemble_steps"], "warmup": len(warm),
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "served", "rate_req_s": args.rate, "duration_s": args.duration,
                   "poisson_frac": args.poisson_frac, "reactor_frac": args.reactor_frac,
                   "budget_gb": args.budget_gb,
                   "poisson_workers": args.poisson_workers,
                   "drain_limit_s": args.drain},
        "served": summary,
    }
    if not args.no_plain:
        ps, _ = serve.serve_plain(trace, time_limit_s=summary["wall_s"], log=log)
        out["plain_form"] = ps
        if ps["throughput_req_s"] > 0:
            out["throughput_ratio_vs_plain"] = summary["throughput_req_s"] / ps["throughput_req_s"]
    print(json.dumps(out))


def bench_reactors(args):
    """Zero-dimensional reactors (the paper's comparison of the reaction algorithm with
    the rate equation): the above-breakdown case, 10^6 reactors of one starting electron
    at 10 MV/m for 50 steps of 1 ps, in one launch of the reactor entry point (inputs
    resident in HBM; HIP events on the context's stream).  Reports reactor-steps/s, the
    ensemble's mean and extinct fraction beside the rate equation's mean and the
    birth-death extinction probability, and the oracle on one host core."""
    import math

    import numpy as np
    import torch

    from paper_2307_01797_amd import itokmc, serve, workloads
    cfg = workloads.preset("reactor_a")
    dev = torch.device("cuda:0")
    sim = serve.reactor_context()
    n, steps, dt = cfg["n_reactors"], cfg["steps"], cfg["dt"]
    k = itokmc.rates(cfg, cfg["E_field"])
    dK = torch.from_numpy(np.tile(k, (n, 1))).to(dev)
    dI = torch.arange(n, dtype=torch.int32, device=dev)
    dF = torch.zeros((n, 5), dtype=torch.int64, device=dev)
    X0 = torch.zeros((n, 4), dtype=torch.int64, device=dev)
    X0[:, 0] = cfg["X0"]
    ms = []
    for rep in range(args.warmup + args.steps):
        dX = X0.clone()
        torch.cuda.synchronize(dev)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(sim.stream)
        sim.kmc_run_device(dI, dX, dK, dt, 100 * rep, steps, dF)
        e1.record(sim.stream)
        torch.cuda.synchronize(dev)
        if rep >= args.warmup:
            ms.append(e0.elapsed_time(e1))
    xe = dX[:, 0].cpu().numpy()
    ka, ke = k[0], k[1]
    r = ka - ke
    g = math.exp(r * steps * dt)
    p0 = ke * (g - 1.0) / (ka * g - ke)
    t_ms = sum(ms) / len(ms)
    out = {
        "metric": "reactor-steps/s (zero-dimensional KMC)",
        "value": n * steps / (t_ms / 1e3), "unit": "reactor-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": t_ms / steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "reactor_a", "reactors": n, "kmc_steps": steps, "dt_s": dt,
                   "E_V_per_m": cfg["E_field"], "X0": cfg["X0"]},
        "statistics": {"mean_e": float(xe.mean()), "rate_equation_mean": cfg["X0"] * g,
                       "extinct_fraction": float((xe == 0).mean()),
                       "birth_death_extinction": p0 ** cfg["X0"]},
    }
    if not args.no_cpu_baseline:
        import oracle
        m = 2_000_000
        X = np.zeros((m, 4), dtype=np.int64)
        X[:, 0] = cfg["X0"]
        K = np.tile(oracle.rates(cfg, cfg["E_field"]), (m, 1))
        t0 = time.perf_counter()
        for s_ in range(steps):
            X, _ = oracle.kmc_cells(cfg, X, K, dt, s_)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": m * steps / el, "unit": "reactor-steps/s", "cores": 1,
                               "kind": "oracle",
                               "sample": f"{m} reactors x {steps} steps in {el:.1f} s"}
    print(json.dumps(out))


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "single-GPU build: this benchmark runs on exactly one GPU; "
                                   "--gpus above 1 is not supported"}))
        sys.exit(2)
    if args.workload.startswith("ensemble"):
        return bench_ensemble(args)
    if args.workload == "reactors":
        return bench_reactors(args)
    if args.workload == "served":
        return bench_served(args)
    import torch

    from paper_2307_01797_amd import itokmc, workloads

    cfg = workloads.preset(args.workload)
    dev = torch.device("cuda:0")
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize(dev)
        del src, dst
    sim = itokmc.Sim(cfg, device=dev)
    sim.seed()
    sim.step(args.warmup)
    torch.cuda.synchronize(dev)
    w = timed_windows(sim, cfg, args.steps, dev)
    for ph, r in w["roofs"].items():
        r["traffic"] = traffic_from_profile(KERNELS[ph], cfg["name"])
        r["valu_busy_pct"] = traffic_from_profile(KERNELS[ph], cfg["name"], "valu_busy_pct")
    roof = max(w["roofs"].values(), key=lambda r: r["total_ms"]) if w["roofs"] else None
    d0, d1, d2 = w["diag"]
    out = {
        "metric": "particle-steps/s (push+sort+deposit+KMC)",
        "value": w["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": w["ms"] / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if cfg.get("precision") == "fp32" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "grid": list(cfg["grid"]), "dx_m": cfg["dx"],
                   "particles_start": d0["n_particles"], "particles_end": d1["n_particles"],
                   "weight_end": d1["weight"], "field": cfg.get("field"),
                   "n_ppc": cfg.get("n_ppc", 0), "dt_s": cfg["dt"], "status": w["rc"],
                   "occupied_cells_end": d2.get("occupied_cells"),
                   "queued_cells_end": d2.get("queued_cells"),
                   "wavefront_coupled_cells_end": d2.get("wave_cells")},
        "profiled_window": {"ms_per_step": w["ms_p"] / args.steps, "status": w["rc_p"],
                            "particle_steps": w["psteps_p"]},
        "phase_ms_per_step": w["phase_ms_per_step"],
        "solver_cycles_per_step": w["cycles"] / args.steps,
        "roofline": roof,
        "roofline_by_kernel": w["roofs"],
    }
    if "push_deposit" in w:
        out["push_deposit"] = w["push_deposit"]
    if cfg.get("field") == "poisson":
        out["dt_rule"] = dt_rule_probe(sim, cfg)
    del sim
    torch.cuda.synchronize(dev)
    if cfg["name"] == "streamer_256" and not args.no_scale_window:
        out["scale_window"] = scale_window(args, dev)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
        if args.cpu_workers > 0:
            out["cpu_baseline_parallel"] = cpu_baseline_parallel(args.cpu_workers, args.cpu_seconds)
    print(json.dumps(out))


def dt_rule_probe(sim, cfg, queries=10):
    """The dynamic time-step rule's field bound on the state the timed windows left:
    `queries` queries (the state is not changed), the per-cell pass timed with HIP
    events; algorithmic bytes per launch = the packed field, 4 S per cell."""
    rule = {"dt_max": cfg["dt"], "c_drift": 0.5, "c_ion": 0.1}
    sim.set_profiling(True)
    sim.phase_times(reset=True)
    for _ in range(queries):
        dt, em = sim.stable_dt(rule)
    tot_ms, launches = sim.phase_times(reset=True)["emax"]
    sim.set_profiling(False)
    ncell = 1
    for v in cfg["grid"]:
        ncell *= v
    S = 8 if cfg.get("precision") == "fp64" else 4
    per_launch = 4 * S * ncell
    achieved = per_launch / (tot_ms / launches / 1e3) / 1e9
    return {"rule": rule, "dt_s": dt, "Emax_V_per_m": em,
            "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                         "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": traffic_from_profile("k_emax_partial", cfg["name"]),
                         "kernel": "k_emax_partial", "avg_launch_ms": round(tot_ms / launches, 4),
                         "launches": launches, "bytes_per_launch": per_launch}}


def push_deposit_roofline(roofs, psteps, S):
    """The particle push with its fused NGP binning and the charge deposit together:
    44 B per particle-step for the push (read cell 4 + offsets 3 x 4 + id 8 + weight 4,
    write cell 4 + offsets 3 x 4) and, in the self-consistent step, 28 B for the
    deposit pass (read cell, offsets, weight and id) plus the particle's mobility that
    the deposit writes and the push reads (2 x 4 B), over the two kernels' time."""
    push = roofs.get("field_push") or roofs.get("push")
    if push is None:
        return None
    dep = roofs.get("deposit")
    per = (20 + 6 * S) + (16 + 3 * S + 2 * S if dep else 0)
    t_ms = push["total_ms"] + (dep["total_ms"] if dep else 0.0)
    achieved = per * psteps / (t_ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "bytes_per_particle_step": per,
            "kernels": [push["kernel"]] + ([dep["kernel"]] if dep else []),
            "ms": round(t_ms, 3), "particle_steps": psteps,
            "particle_steps_per_s": psteps / (t_ms / 1e3)}


def timed_windows(sim, cfg, steps, dev):
    """K timed steps (HIP events on the library's stream), then K profiled steps (HIP
    events around every kernel phase): the rate, the per-phase times, the roofline of
    each single-kernel phase."""
    import torch
    stream = sim.stream
    d0 = sim.diagnostics()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize(dev)
    ev0.record(stream)
    rc = sim.step_rc(steps)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    ms = ev0.elapsed_time(ev1)
    d1 = sim.diagnostics(check=False)
    psteps = d1["particle_steps"] - d0["particle_steps"]
    # profiled window: the next K steps with HIP events around every kernel phase (and
    # around each finest-level smoother launch, whose cycles then run without the graph)
    sim.set_profiling(True)
    sim.phase_times(reset=True)
    ev0.record(stream)
    rc_p = sim.step_rc(steps)
    ev1.record(stream)
    torch.cuda.synchronize(dev)
    ms_p = ev0.elapsed_time(ev1)
    phases = sim.phase_times(reset=True)
    sim.set_profiling(False)
    d2 = sim.diagnostics(check=False)
    psteps_p = d2["particle_steps"] - d1["particle_steps"]
    ncell = 1
    for v in cfg["grid"]:
        ncell *= v
    S = 8 if cfg.get("precision") == "fp64" else 4
    roofs = {}
    for ph, kname in KERNELS.items():
        tot_ms, launches = phases.get(ph, (0.0, 0))
        if not launches or tot_ms <= 0:
            continue
        if ph in ("smooth_fine", "ions"):
            units = ncell * launches
        elif ph == "couple":
            units = d2.get("couple_pieces", 0) - d1.get("couple_pieces", 0)
        else:
            units = psteps_p
        per_unit = bytes_per_unit(ph, S)
        if ph == "couple" and not cfg.get("n_ppc", 0):
            per_unit = 12
        per_launch = per_unit * units / launches
        achieved = per_launch / (tot_ms / launches / 1e3) / 1e9
        roofs[ph] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": kname if ph != "ions" else "k_ion_clear, k_ion_move, k_ion_commit",
                     "avg_launch_ms": round(tot_ms / launches, 4),
                     "launches": launches, "bytes_per_launch": int(per_launch),
                     "total_ms": round(tot_ms, 3)}
    out = {"value": psteps / (ms / 1e3), "ms": ms, "rc": rc, "ms_p": ms_p, "rc_p": rc_p,
           "psteps": psteps, "psteps_p": psteps_p, "diag": (d0, d1, d2), "roofs": roofs,
           "phase_ms_per_step": {p: round(v[0] / steps, 4) for p, v in phases.items() if v[1]},
           "cycles": d1.get("solver_cycles_total", 0) - d0.get("solver_cycles_total", 0)}
    pd = push_deposit_roofline(roofs, psteps_p, S)
    if pd is not None:
        out["push_deposit"] = pd
    return out


def scale_window(args, dev):
    """The self-consistent streamer near the configuration's particle cap (the denser
    seed of workloads.STREAMER_256_DENSE, about 4.4e7 particles after the first
    superparticle pass): two warm-up steps, then a timed and a profiled window."""
    import torch

    from paper_2307_01797_amd import itokmc, workloads
    cfg = workloads.preset("streamer_256_dense")
    sim = itokmc.Sim(cfg, device=dev)
    sim.seed()
    sim.step(2)
    torch.cuda.synchronize(dev)
    w = timed_windows(sim, cfg, args.scale_steps, dev)
    d0, d1, _ = w["diag"]
    res = {"workload": cfg["name"], "steps": args.scale_steps, "warmup": 2,
           "particles_start": d0["n_particles"], "particles_end": d1["n_particles"],
           "value": w["value"], "unit": "particle-steps/s",
           "ms_per_step": w["ms"] / args.scale_steps, "status": w["rc"],
           "phase_ms_per_step": w["phase_ms_per_step"],
           "roofline_by_kernel": w["roofs"]}
    if "push_deposit" in w:
        res["push_deposit"] = w["push_deposit"]
    del sim
    torch.cuda.synchronize(dev)
    return res


if __name__ == "__main__":
    main()
