"""Batched and served forms of the method on one GPU, over the itokmc C ABI.

* run_batched: a fixed set of uniform-field realizations admitted into one batched
  ensemble and stepped together until every one is done.
* run_plain: the same realizations one at a time, each in its own single context
  (the plain per-realization form).
* Server: a request loop with continuous batching.  Uniform-field requests are
  admitted into the resident ensemble as soon as a slot, pool cells and particle quota
  are free (the arena is sized from an HBM budget); each ensemble step advances every
  resident request, and finished ones are reported and released between steps while
  new ones join.  Self-consistent (Poisson) requests run in single contexts on worker
  threads with streams of their own, admitted against the remaining budget, so their
  kernels overlap the ensemble's on the device.
* Zero-dimensional reactor requests (ensembles of independent reactors, the paper's
  comparison of the reaction algorithm with the rate equation) are gathered between
  ensemble steps and run together in one launch of the library's reactor entry point
  on a stream of their own; each reactor keeps its request's key and its own stream,
  so a request's result does not depend on what it was batched with.
* serve_plain: the same request stream handled first-come first-served, one request
  at a time in single contexts.

Every request's stop rule is the library's: a request is done after its step budget
or after the first step that began with at least stop_particles live particles.
Host code here only schedules; all arithmetic runs in the library's kernels.
"""
import collections
import queue
import threading
import time

import numpy as np

from . import itokmc

BANK_BYTES_FP32 = 2 * 32   # both particle banks, bytes per particle slot
CELL_BYTES = 36            # ensemble per-cell arrays


def _stop_rule_run(sim, cfg, cancelled=None):
    """Step a single context under the stop rule, evaluated on the device
    (itokmc_step_until: one call; in the self-consistent mode the host reads the
    device's decision after each step, whose field solve synchronises anyway); returns
    steps run, or None if cancelled() was already true."""
    if cancelled is not None and cancelled():
        return None
    return sim.step_until(int(cfg["steps"]), int(cfg.get("stop_particles", 0)))


def run_plain_one(cfg, device="cuda:0", stream=None, keep_particles=False, cancelled=None):
    """One request in its own context; returns (diagnostics, particles or None), or
    (None, None) if cancelled."""
    sim = itokmc.Sim(cfg, device=device, max_particles=cfg["max_particles"], stream=stream)
    try:
        sim.seed()
        if _stop_rule_run(sim, cfg, cancelled) is None:
            return None, None
        d = sim.diagnostics(check=False)
        parts = sim.particles() if keep_particles else None
        return d, parts
    finally:
        sim.close()


def run_plain(cfgs, device="cuda:0", log=None):
    """Plain per-realization form: each realization alone, one after another.
    log: optional callable receiving a progress line now and then."""
    import torch
    dev = torch.device(device)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    results = []
    for i, c in enumerate(cfgs):
        results.append(run_plain_one(c, device)[0])
        if log and (i + 1) % 32 == 0:
            log(f"plain form: {i + 1}/{len(cfgs)} realizations, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize(dev)
    sec = time.perf_counter() - t0
    return dict(seconds=sec, results=results,
                particle_steps=sum(r["particle_steps"] for r in results))


def ensemble_for(cfgs, max_slots=None, device="cuda:0"):
    """An ensemble whose pools hold all of cfgs at once."""
    blocks = sum(-(-int(np.prod(c["grid"])) // 4096) for c in cfgs)
    quota = sum(int(c["max_particles"]) for c in cfgs)
    return itokmc.Ensemble(max_slots or len(cfgs), blocks * 4096, quota,
                           precision=cfgs[0].get("precision", "fp32"), device=device)


def run_batched(cfgs, ens=None, steps_per_poll=2, device="cuda:0"):
    """Batched form: admit every realization, step the ensemble, and collect and
    release realizations as they finish (their particles leave the pool at the next
    step) until all are done."""
    import torch
    dev = torch.device(device)
    ens = ens or ensemble_for(cfgs, device=device)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    for i, c in enumerate(cfgs):
        if ens.admit(c, tag=i) is None:
            raise RuntimeError("ensemble pools too small for the batch")
    results = [None] * len(cfgs)
    left = len(cfgs)
    while left:
        ens.step(steps_per_poll)
        events = ens.poll()
        if events:
            diags = ens.results([e[0] for e in events])
            for (slot, state, tag, steps), d in zip(events, diags):
                d["state"] = state
                results[tag] = d
                ens.release(slot)
            left -= len(events)
    torch.cuda.synchronize(dev)
    sec = time.perf_counter() - t0
    ens.step(1)  # drop the last released realizations' particles
    return dict(seconds=sec, results=results, ensemble=ens,
                particle_steps=sum(r["particle_steps"] for r in results))


def reactor_context(device="cuda:0", stream=None):
    """A small context whose method parameters (hybrid KMC, seed 1) the reactor lane
    uses; each reactor brings its own realization (key) and rates."""
    from . import workloads
    return itokmc.Sim(workloads.REACTOR_A, device=device, stream=stream, max_particles=1024)


def run_reactors(sim, cfgs, keep=False):
    """Run reactor requests (equal dt) in one launch: reactor j of request r starts with
    X0 electrons, takes the request's rates at its field and its step count, under the
    key (seed, r) and stream cell id j.  Returns per request the mean and the number
    of extinct final electron counts, the fire totals, and (keep) the final counts."""
    torch = sim.torch
    dt = cfgs[0]["dt"]
    assert all(c["dt"] == dt for c in cfgs)
    n = [int(c["n_reactors"]) for c in cfgs]
    N = sum(n)
    X = np.zeros((N, 4), dtype=np.int64)
    K = np.zeros((N, 5))
    ids = np.zeros(N, dtype=np.int32)
    real = np.zeros(N, dtype=np.int32)
    steps = np.zeros(N, dtype=np.int32)
    o = 0
    for c, m in zip(cfgs, n):
        X[o:o + m, 0] = c["X0"]
        K[o:o + m] = itokmc.rates(c, c["E_field"])
        ids[o:o + m] = np.arange(m, dtype=np.int32)
        real[o:o + m] = np.int32(np.uint32(c["realization"]).view(np.int32))
        steps[o:o + m] = c["steps"]
        o += m
    dev = sim.device
    dX = torch.from_numpy(X).to(dev)
    dK = torch.from_numpy(K).to(dev)
    dI = torch.from_numpy(ids).to(dev)
    dR = torch.from_numpy(real).to(dev)
    dS = torch.from_numpy(steps).to(dev)
    dF = torch.zeros((N, 5), dtype=torch.int64, device=dev)
    sim.stream.synchronize()
    sim.kmc_run_device(dI, dX, dK, dt, 0, 0, dF, realization=dR, steps=dS)
    sim.stream.synchronize()
    Xh = dX.cpu().numpy()
    Fh = dF.cpu().numpy()
    out = []
    o = 0
    for c, m in zip(cfgs, n):
        xe = Xh[o:o + m, 0]
        out.append(dict(n=m, mean_e=float(xe.mean()), extinct=int((xe == 0).sum()),
                        fires=[int(v) for v in Fh[o:o + m].sum(axis=0)],
                        reactor_steps=m * int(c["steps"]),
                        final=Xh[o:o + m].copy() if keep else None))
        o += m
    return out


def _percentiles(lat):
    if not lat:
        return None, None
    a = np.sort(np.asarray(lat))
    return float(np.percentile(a, 50)), float(np.percentile(a, 99))


class Server:
    """Continuous-batching request loop on one GPU (see the module docstring).

    budget_bytes: device memory the service may hold; the ensemble arena takes
    (1 - poisson_share) of it, self-consistent requests reserve their context arenas
    from the rest.  keep: request ids whose final particles are returned."""

    def __init__(self, budget_bytes=200e9, max_slots=1024, poisson_share=0.25,
                 poisson_workers=2, slot_particles=1_250_000, slot_cells=96**3,
                 device="cuda:0", keep=()):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        ens_budget = budget_bytes * (1.0 - poisson_share)
        per_slot = slot_particles * BANK_BYTES_FP32 + slot_cells * CELL_BYTES
        slots = int(max(1, min(max_slots, ens_budget // per_slot)))
        cells = -(-slots * slot_cells // 4096) * 4096
        particles = min(0x7FFFFFFF, slots * slot_particles)
        self.ens = itokmc.Ensemble(slots, cells, particles, device=device)
        self.slots = slots
        self.budget = budget_bytes
        self.poisson_budget = max(0.0, budget_bytes - self.ens.arena_bytes)
        self.poisson_free = self.poisson_budget
        self.poisson_workers = poisson_workers
        self.keep = set(keep)
        self.cv = threading.Condition()
        self._cancel = threading.Event()
        self.reactor_stream = torch.cuda.Stream(self.device)
        self.reactors = reactor_context(device, self.reactor_stream)

    # -- self-consistent lane -------------------------------------------------------
    def _poisson_worker(self, q, results, t0, stream, errors):
        torch = self.torch
        cancelled = self._cancel.is_set
        try:
            with torch.cuda.stream(stream):
                while not cancelled():
                    try:
                        item = q.get(timeout=0.05)
                    except queue.Empty:
                        continue
                    if item is None:
                        return
                    t_arr, rid, cfg = item
                    need = itokmc.arena_bytes(cfg, max_particles=cfg["max_particles"])
                    if need > self.poisson_budget:
                        results[rid] = dict(kind="poisson", arrival=t_arr, rejected=True)
                        continue
                    with self.cv:
                        while self.poisson_free < need and not cancelled():
                            self.cv.wait(0.05)
                        if cancelled():
                            return
                        self.poisson_free -= need
                    t_adm = time.perf_counter() - t0
                    try:
                        d, parts = run_plain_one(cfg, self.device, stream, rid in self.keep,
                                                 cancelled)
                    finally:
                        with self.cv:
                            self.poisson_free += need
                            self.cv.notify_all()
                    if d is None:
                        return
                    results[rid] = dict(kind="poisson", arrival=t_arr, admitted=t_adm,
                                        finished=time.perf_counter() - t0, diag=d,
                                        particles=parts)
        except Exception as e:  # reported by run()
            errors.append(repr(e))

    # -- main loop ----------------------------------------------------------------------
    def run(self, trace, drain_limit_s=None, steps_per_poll=1, log=None):
        """Serve a request trace [(arrival_s, id, cfg)] in real time.  Returns a summary
        and the per-request records (arrival, admission and finish times in s).
        log: optional callable receiving a progress line every 10 s."""
        torch = self.torch
        ens = self.ens
        results = {}
        errors = []
        pq = queue.Queue()
        streams = [torch.cuda.Stream(self.device) for _ in range(self.poisson_workers)]
        torch.cuda.synchronize(self.device)
        t0 = time.perf_counter()
        workers = [threading.Thread(target=self._poisson_worker, args=(pq, results, t0, s, errors),
                                    daemon=True) for s in streams]
        for w in workers:
            w.start()
        end_arrivals = trace[-1][0] if trace else 0.0
        i = 0
        pending = collections.deque()
        rq = []   # reactor requests waiting for the next batch
        active = {}
        batched_steps = 0
        max_active = 0
        self.admission_waits = 0
        next_log = 10.0
        while True:
            now = time.perf_counter() - t0
            if log and now >= next_log:
                next_log += 10.0
                log(f"served: t={now:.0f} s arrived {i}/{len(trace)} resident {len(active)} "
                    f"queued {len(pending)} done {len(results)}")
            while i < len(trace) and trace[i][0] <= now:
                item = trace[i]
                i += 1
                if item[2].get("kind") == "reactor":
                    rq.append(item)
                elif item[2].get("field") == "poisson":
                    pq.put(item)
                else:
                    pending.append(item)
            while pending:
                t_arr, rid, cfg = pending[0]
                slot = ens.admit(cfg, tag=rid)
                if slot is None and not active:
                    ens.step(1)  # an empty step returns released cells and quota
                    slot = ens.admit(cfg, tag=rid)
                    if slot is None:
                        # larger than the whole ensemble: can never be admitted
                        pending.popleft()
                        results[rid] = dict(kind="batched", arrival=t_arr, rejected=True)
                        continue
                if slot is None:
                    self.admission_waits += 1
                    break
                pending.popleft()
                active[slot] = (rid, t_arr, now)
            max_active = max(max_active, len(active))
            if rq:
                # reactor requests: one launch per time step length, overlapping the
                # ensemble's queued work on the device
                t_adm = time.perf_counter() - t0
                by_dt = collections.defaultdict(list)
                for item in rq:
                    by_dt[item[2]["dt"]].append(item)
                rq = []
                for items in by_dt.values():
                    outs = run_reactors(self.reactors, [c for _, _, c in items],
                                        keep=any(rid in self.keep for _, rid, _ in items))
                    tf = time.perf_counter() - t0
                    for (t_arr, rid, cfg), res in zip(items, outs):
                        if rid not in self.keep:
                            res["final"] = None
                        results[rid] = dict(kind="reactor", arrival=t_arr, admitted=t_adm,
                                            finished=tf, reactor=res)
            if active:
                ens.step(steps_per_poll)
                batched_steps += steps_per_poll
                events = ens.poll()
                tf = time.perf_counter() - t0
                diags = ens.results([e[0] for e in events]) if events else []
                for (slot, state, tag, steps), d in zip(events, diags):
                    rid, t_arr, t_adm = active.pop(slot)
                    parts = ens.particles(slot) if rid in self.keep else None
                    ens.release(slot)
                    results[rid] = dict(kind="batched", arrival=t_arr, admitted=t_adm,
                                        finished=tf, state=state, steps=steps, diag=d,
                                        particles=parts)
            elif i >= len(trace) and not pending and not rq:
                break
            elif i < len(trace):
                time.sleep(max(0.0, min(0.002, trace[i][0] - now)))
            if drain_limit_s is not None and now > end_arrivals + drain_limit_s:
                break
        # let the self-consistent lane finish its queue, within the drain limit
        for _ in workers:
            pq.put(None)
        deadline = None if drain_limit_s is None else t0 + end_arrivals + drain_limit_s
        last = time.perf_counter()
        for w in workers:
            while w.is_alive():
                w.join(0.1)
                if deadline is not None and time.perf_counter() > deadline:
                    self._cancel.set()
                if log and time.perf_counter() - last > 10.0:
                    last = time.perf_counter()
                    log(f"served: draining self-consistent lane, done {len(results)}")
        torch.cuda.synchronize(self.device)
        if errors:
            raise RuntimeError("self-consistent worker failed: " + "; ".join(errors))
        wall = time.perf_counter() - t0
        return self._summary(trace, results, wall, batched_steps, max_active), results

    def _summary(self, trace, results, wall, batched_steps, max_active):
        lat_all, lat_b, lat_p, lat_r = [], [], [], []
        psteps = 0
        rsteps = 0
        done = 0
        unfinished_poisson = 0
        for t, rid, cfg in trace:
            r = results.get(rid)
            if r is None or r.get("rejected"):
                if cfg.get("field") == "poisson":
                    unfinished_poisson += 1
                continue
            done += 1
            lat = r["finished"] - r["arrival"]
            lat_all.append(lat)
            if r["kind"] == "reactor":
                lat_r.append(lat)
                rsteps += r["reactor"]["reactor_steps"]
                continue
            (lat_p if r["kind"] == "poisson" else lat_b).append(lat)
            psteps += r["diag"]["particle_steps"]
        p50, p99 = _percentiles(lat_all)
        b50, b99 = _percentiles(lat_b)
        q50, q99 = _percentiles(lat_p)
        r50, r99 = _percentiles(lat_r)
        n = len(trace)
        return dict(requests=n, completed=done, unfinished=n - done,
                    unfinished_poisson=unfinished_poisson, wall_s=wall,
                    throughput_req_s=done / wall if wall > 0 else 0.0,
                    particle_steps_per_s=psteps / wall if wall > 0 else 0.0,
                    p50_s=p50, p99_s=p99, batched_p50_s=b50, batched_p99_s=b99,
                    poisson_p50_s=q50, poisson_p99_s=q99, reactor_p50_s=r50,
                    reactor_p99_s=r99, reactor_requests=len(lat_r),
                    reactor_steps_per_s=rsteps / wall if wall > 0 else 0.0, slots=self.slots,
                    max_resident=max_active, ensemble_steps=batched_steps,
                    admission_waits=self.admission_waits,
                    ensemble_arena_gb=self.ens.arena_bytes / 1e9)


def serve_plain(trace, time_limit_s, device="cuda:0", keep=(), log=None):
    """First-come first-served, one request at a time in a single context; stops
    starting new requests after time_limit_s.  Returns (summary, records)."""
    import torch
    dev = torch.device(device)
    torch.cuda.synchronize(dev)
    t0 = time.perf_counter()
    results = {}
    psteps = 0
    next_log = 10.0
    reactors = None
    for t_arr, rid, cfg in trace:
        now = time.perf_counter() - t0
        if now > time_limit_s:
            break
        if log and now >= next_log:
            next_log += 10.0
            log(f"plain serving: t={now:.0f} s done {len(results)}")
        if t_arr > now:
            time.sleep(t_arr - now)
        t_adm = time.perf_counter() - t0
        if cfg.get("kind") == "reactor":
            if reactors is None:
                reactors = reactor_context(device)
            res = run_reactors(reactors, [cfg], keep=rid in keep)[0]
            results[rid] = dict(kind="reactor", arrival=t_arr, admitted=t_adm,
                                finished=time.perf_counter() - t0, reactor=res)
            continue
        d, parts = run_plain_one(cfg, device, keep_particles=rid in keep)
        results[rid] = dict(kind=cfg.get("field", "uniform"), arrival=t_arr, admitted=t_adm,
                            finished=time.perf_counter() - t0, diag=d, particles=parts)
        psteps += d["particle_steps"]
    torch.cuda.synchronize(dev)
    wall = time.perf_counter() - t0
    lat = [r["finished"] - r["arrival"] for r in results.values()]
    p50, p99 = _percentiles(lat)
    return dict(requests=len(trace), completed=len(results),
                unfinished=len(trace) - len(results), wall_s=wall,
                throughput_req_s=len(results) / wall if wall > 0 else 0.0,
                particle_steps_per_s=psteps / wall if wall > 0 else 0.0,
                p50_s=p50, p99_s=p99), results
