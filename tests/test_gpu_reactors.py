"""Zero-dimensional reactors (the paper's comparison of the reaction algorithm with the
rate equation; itokmc_kmc_run): many independent reactors of ionization and attachment
stepped in one launch.

* Parity: every reactor's final populations and fire totals equal the oracle's, step by
  step on the same streams, for several requests (keys, fields, starting counts, step
  counts) batched in one launch; a request's result is the same alone and batched.
* At scale, against closed forms of the linear birth-death process (rates k_a, k_e,
  r = k_a - k_e): the mean X0 exp(r t) of the rate equation and the extinction
  probability P0(t) = k_e (e^{rt} - 1) / (k_a e^{rt} - k_e) per starting electron, for
  the paper's two cases: above breakdown (10 MV/m, one electron, 50 ps) and below
  breakdown (1.7 MV/m, five electrons, 50 ns, where all five attach in most reactors
  while the rate equation keeps a fractional electron).
* Served: reactor requests arriving among batched avalanches give the same results as
  run alone.
"""
import math

import numpy as np
import pytest

from paper_2307_01797_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def serve():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2307_01797_amd import itokmc, serve as s
    itokmc.lib()
    return s


@pytest.fixture(scope="module")
def ctx(serve):
    return serve.reactor_context()


def _oracle_reactors(orc, cfg):
    n = cfg["n_reactors"]
    X = np.zeros((n, 4), dtype=np.int64)
    X[:, 0] = cfg["X0"]
    k = np.tile(orc.rates(cfg, cfg["E_field"]), (n, 1))
    F = np.zeros((n, 5), dtype=np.int64)
    for s in range(cfg["steps"]):
        X, f = orc.kmc_cells(cfg, X, k, cfg["dt"], s)
        F += f
    return X, F


def test_reactors_match_oracle_and_batching(serve, ctx, orc):
    cfgs = [dict(workloads.reactor_request(r), n_reactors=1500, steps=s)
            for r, s in ((3, 40), (11, 25), (20, 60))]
    cfgs[0].update(E_field=1.0e7, X0=1)
    cfgs[1].update(E_field=1.2e7, X0=80)    # leaps: A dt > 1 for most of the run
    cfgs[2].update(E_field=2.0e6, X0=3)     # attachment dominated, critical (X_e < 5)
    batch = serve.run_reactors(ctx, cfgs, keep=True)
    for cfg, res in zip(cfgs, batch):
        X, F = _oracle_reactors(orc, cfg)
        assert np.array_equal(res["final"], X), cfg["name"]
        assert res["fires"] == [int(v) for v in F.sum(axis=0)]
        alone = serve.run_reactors(ctx, [cfg], keep=True)[0]
        assert np.array_equal(alone["final"], res["final"])
    assert batch[1]["fires"][0] > 1000 and batch[2]["fires"][1] > 0


def _birth_death(cfg, orc):
    k = orc.rates(cfg, cfg["E_field"])
    ka, ke = k[0], k[1]
    r = ka - ke
    t = cfg["steps"] * cfg["dt"]
    g = math.exp(r * t)
    p0 = ke * (g - 1.0) / (ka * g - ke)
    var1 = (ka + ke) / r * g * (g - 1.0)   # variance per starting electron
    return g, p0, var1


@pytest.mark.parametrize("case", ["reactor_a", "reactor_b"])
def test_reactor_statistics_match_closed_forms(serve, ctx, orc, case):
    cfg = workloads.preset(case)
    res = serve.run_reactors(ctx, [cfg], keep=True)[0]
    n, X0 = cfg["n_reactors"], cfg["X0"]
    g, p0, var1 = _birth_death(cfg, orc)
    xe = res["final"][:, 0]
    # mean against the rate equation X0 exp(r t)
    se = math.sqrt(X0 * var1 / n)
    assert abs(xe.mean() - X0 * g) < 5 * se, (xe.mean(), X0 * g, se)
    # extinction: all X0 lineages die out independently
    pe = p0 ** X0
    se_p = math.sqrt(pe * (1 - pe) / n)
    assert abs((xe == 0).mean() - pe) < 5 * se_p, ((xe == 0).mean(), pe)
    # charge: -e + M+ - M- is invariant in every reactor
    f = res["final"]
    assert np.all(-f[:, 0] + f[:, 1] - f[:, 2] == -X0)
    if case == "reactor_a":
        assert g == pytest.approx(1.916, rel=1e-3) and p0 == pytest.approx(0.01514, rel=1e-3)
    else:
        # below breakdown the rate equation keeps a fraction of an electron while most
        # reactors lose all five
        assert X0 * g < 0.1 and (xe == 0).mean() > 0.9


def test_served_reactors_match_alone(serve):
    tr = workloads.request_trace(rate=400.0, duration=10.0, poisson_frac=0.0, seed=7,
                                 reactor_frac=0.5)[:24]
    trace = []
    for t, rid, c in tr:
        c = dict(c)
        if c.get("kind") == "reactor":
            c["steps"] = min(c["steps"], 80)
        else:
            L = 32 * c["dx"]
            c.update(grid=(32, 32, 32), seed_centre=(L / 2,) * 3, seed_sigma=0.156 * L,
                     seed_n0=min(c["seed_n0"], 2000), steps=30, stop_particles=4500,
                     max_particles=300_000)
        trace.append((t, rid, c))
    kinds = [c.get("kind") for _, _, c in trace]
    assert kinds.count("reactor") >= 6 and kinds.count(None) >= 6
    srv = serve.Server(budget_bytes=2.0e9, max_slots=6, poisson_share=0.0, poisson_workers=1,
                       slot_particles=300_000, slot_cells=48**3, keep=[t[1] for t in trace])
    summary, recs = srv.run(trace)
    assert summary["completed"] == len(trace)
    assert summary["reactor_requests"] == kinds.count("reactor")
    ctx = serve.reactor_context()
    for t, rid, cfg in trace:
        if cfg.get("kind") != "reactor":
            continue
        alone = serve.run_reactors(ctx, [cfg], keep=True)[0]
        assert np.array_equal(recs[rid]["reactor"]["final"], alone["final"])
        assert recs[rid]["reactor"]["fires"] == alone["fires"]
