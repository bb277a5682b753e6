"""Pins of the oracle's recombination chemistry (rows 3 and 4 of the paper's air
table: e + M+ -> 0 with propensity k_ep X_e X_M+, M- + M+ -> 0 with k_np X_M+ X_M-;
rates of the section "Simulation conditions"; the step-4 factor g_i of the reaction
algorithm outline).  Each pin is a law the mathematics fixes:
  - rate values at the gas temperature and the T_e power law;
  - the exact distribution of each recombination death chain (master equation,
    solved by matrix exponential) in the SSA regime and in the critical regime;
  - Cao's leap condition: over the selected leap, no non-critical propensity changes
    by a relative amount above eps (first order in the mean and the standard
    deviation), with equality for the binding species;
  - the rate-equation solution n(t) = n0 / (1 + k n0 t) for a large population leapt
    with a small eps (and a visibly worse one-leap answer with eps = inf);
  - charge conservation and ion-only cells in full steps."""
import math

import numpy as np
import pytest
from scipy import linalg, stats

from paper_2307_01797_amd import workloads

DT = 1e-12


def _cfg(**kw):
    return workloads.preset("avalanche_32", **kw)


def test_rates_at_gas_temperature_and_power_law(orc):
    cfg = _cfg(coeffs=workloads.RECOMBINATION)
    dV = cfg["dx"] ** 3
    # E at the floor: T_e = max(300 K, 1e4 K * 0.01^0.5 = 1000 K) = 1000 K
    k = orc.rates(cfg, 0.0)
    assert k[3] * dV == pytest.approx(1.138e-11 * 1000.0 ** -0.7, rel=1e-12)
    assert k[3] * dV == pytest.approx(9.0395e-14, rel=1e-4)
    assert k[4] * dV == pytest.approx(2.0e-13, rel=1e-15)
    # T_e = 1e4 sqrt(E / 1 MV/m): quadrupling E doubles T_e, beta_ep falls by 2^-0.7
    r = orc.rates(cfg, 4e7)[3] / orc.rates(cfg, 1e7)[3]
    assert r == pytest.approx(2.0 ** -0.7, rel=1e-12)
    # the 300 K floor: a field-free cell with a tiny Te_a sits at the gas temperature
    cold = _cfg(coeffs=dict(workloads.RECOMBINATION, Te_a=1.0))
    assert orc.rates(cold, 0.0)[3] * dV == pytest.approx(1.138e-11 * 300.0 ** -0.7, rel=1e-12)
    # off when absent
    assert orc.rates(_cfg(), 1e7)[3] == 0.0 and orc.rates(_cfg(), 1e7)[4] == 0.0


def _death_chain_law(n0, delta, kdt, steps):
    """P(n) after steps*dt for the chain n -> n-1 at rate k n (n + delta)."""
    Q = np.zeros((n0 + 1, n0 + 1))
    for n in range(1, n0 + 1):
        q = kdt * n * (n + delta)
        Q[n, n] -= q
        Q[n, n - 1] += q
    p0 = np.zeros(n0 + 1)
    p0[n0] = 1.0
    return p0 @ linalg.expm(Q * steps)


def _chisq(obs, p, n):
    exp = n * p
    keep = exp >= 10
    o = np.append(obs[keep], obs[~keep].sum())
    e = np.append(exp[keep], exp[~keep].sum())
    if e[-1] < 1e-9:
        o, e = o[:-1], e[:-1]
    e = e * o.sum() / e.sum()
    return stats.chisquare(o, e).pvalue


def _run(orc, cfg, X0, k5, steps, n):
    X = np.tile(np.asarray(X0, dtype=np.int64), (n, 1))
    K = np.tile(np.asarray(k5, dtype=np.float64), (n, 1))
    F = np.zeros((n, 5), dtype=np.int64)
    for s in range(steps):
        X, f = orc.kmc_cells(cfg, X, K, DT, s)
        F += f
        assert X.min() >= 0
        assert np.all(-X[:, 0] + X[:, 1] - X[:, 2] == -X0[0] + X0[1] - X0[2])
    return X, F


@pytest.mark.parametrize("n0,delta,adt,steps", [(30, 5, 1.0, 40), (4, 2, 40.0, 1)])
def test_electron_ion_recombination_master_equation(orc, n0, delta, adt, steps):
    """e + M+ -> 0 alone: X_e is a death chain with rate k n (n + delta).  With
    A dt <= 1 every pass is the SSA exception; with X_e < N_c the reaction is critical
    and fires one event at a time (branch 6(a)); both are exact."""
    kdt = adt / (n0 * (n0 + delta))
    n = 20000
    X, F = _run(orc, _cfg(), [n0, n0 + delta, 0, 0], [0, 0, 0, kdt / DT, 0], steps, n)
    assert np.array_equal(X[:, 1] - X[:, 0], np.full(n, delta))
    assert np.array_equal(F[:, 3], n0 - X[:, 0]) and F[:, :3].sum() == 0 and F[:, 4].sum() == 0
    p = _death_chain_law(n0, delta, kdt, steps)
    assert _chisq(np.bincount(X[:, 0], minlength=n0 + 1), p, n) > 1e-4
    # the law separates a mistaken propensity (k n^2: the extra ions ignored)
    q = _death_chain_law(n0, 0, kdt, steps)
    assert abs(p @ np.arange(n0 + 1) - q @ np.arange(n0 + 1)) > 0.05


def test_ion_ion_recombination_master_equation(orc):
    """M- + M+ -> 0 alone in a cell with no electrons: X_M- is a death chain with rate
    k m (m + delta), delta = X_M+ - X_M-."""
    n0, delta, steps = 25, 8, 30
    kdt = 1.0 / (n0 * (n0 + delta))
    n = 20000
    X, F = _run(orc, _cfg(), [0, n0 + delta, n0, 0], [0, 0, 0, 0, kdt / DT], steps, n)
    assert np.array_equal(X[:, 1] - X[:, 2], np.full(n, delta)) and X[:, 0].max() == 0
    assert np.array_equal(F[:, 4], n0 - X[:, 2])
    p = _death_chain_law(n0, delta, kdt, steps)
    assert _chisq(np.bincount(X[:, 2], minlength=n0 + 1), p, n) > 1e-4


def _leap_checks(orc, cfg, X, k, eps):
    """First-order relative change of each non-critical propensity over the leap."""
    tau = orc.kmc_leap_bound(cfg, X, k)
    a = np.array([k[0] * X[0], k[1] * X[0], k[2] * X[0], k[3] * X[0] * X[1], k[4] * X[1] * X[2]])
    nu = np.array([[1, 1, 0, 0], [-1, 0, 1, 0], [0, 0, 0, 1], [-1, -1, 0, 0], [0, -1, -1, 0]])
    react = [[0], [0], [0], [0, 1], [1, 2]]
    nc = 5
    crit = [any(nu[r, i] < 0 and X[i] < nc for i in range(4)) for r in range(5)]
    live = [r for r in range(5) if k[r] > 0 and not crit[r]]
    mean = sum(nu[r] * a[r] for r in live) * tau          # E[dX] over the leap
    sd = np.sqrt(sum(nu[r] ** 2 * a[r] for r in live) * tau)
    worst_mean = max(sum(abs(mean[i]) / X[i] for i in react[r]) for r in live)
    worst_sd = max(sum(sd[i] / X[i] for i in react[r]) for r in live)
    return tau, worst_mean, worst_sd


def test_leap_bound_keeps_propensity_change_below_eps(orc):
    """Step 4's purpose: over the chosen leap no non-critical propensity changes by a
    relative amount above eps.  A second-order propensity k X_i X_j changes by the sum
    of its reactants' relative changes, which is why g_i = 2 for their species; with
    g_i = 1 the recombination propensities would change by up to 2 eps."""
    eps = 0.03
    cfg = _cfg(kmc_eps=eps)
    rng = np.random.default_rng(7)
    binding = 0
    for _ in range(300):
        X = np.array([rng.integers(2000, 200000), rng.integers(2000, 200000),
                      rng.integers(2000, 200000), 0], dtype=np.int64)
        k = np.array([rng.uniform(0, 2e10), rng.uniform(0, 1e10), rng.uniform(0, 1e9),
                      10 ** rng.uniform(0, 6), 10 ** rng.uniform(0, 6)])
        tau, wm, ws = _leap_checks(orc, cfg, X, k, eps)
        assert 0 < tau < math.inf
        assert wm <= eps * (1 + 1e-9) and ws <= eps * (1 + 1e-9)
        binding += max(wm, ws) > 0.5 * eps
    assert binding > 250        # the bound is not slack: some propensity is near eps
    # first-order network only (recombination off): g = 1, the electron propensities
    # reach eps on their own
    X = np.array([50000, 80000, 1000, 0], dtype=np.int64)
    tau1 = orc.kmc_leap_bound(cfg, X, [1.3e10, 4e8, 0, 0, 0])
    tau2 = orc.kmc_leap_bound(cfg, X, [1.3e10, 4e8, 0, 1e-30, 0])
    mean_e = (1.3e10 - 4e8) * X[0]
    assert tau1 * mean_e / X[0] == pytest.approx(eps, rel=1e-12)
    assert tau2 == pytest.approx(tau1 / 2, rel=1e-12)   # e joins a second-order reaction
    assert orc.kmc_leap_bound(_cfg(), X, [1.3e10, 4e8, 0, 1.0, 1.0]) == math.inf


def test_large_population_follows_rate_equation(orc):
    """e + M+ -> 0 with X_e = X_M+ = n0 = 1e5: the rate equation dn/dt = -k n^2 gives
    n(dt) = n0 / (1 + k n0 dt) = n0 / 1.5.  Leaps bounded by eps = 0.02 reproduce it to
    well under 1%; a single unbounded leap (eps = inf) does not."""
    n0 = 100000
    k = 0.5 / (n0 * DT)
    want = n0 / 1.5
    n = 200
    X, _ = _run(orc, _cfg(kmc_eps=0.02), [n0, n0, 0, 0], [0, 0, 0, k, 0], 1, n)
    assert abs(X[:, 0].mean() / want - 1) < 5e-3
    Xi, _ = _run(orc, _cfg(), [n0, n0, 0, 0], [0, 0, 0, k, 0], 1, n)
    assert abs(Xi[:, 0].mean() / want - 1) > 0.1


def _recomb_coeffs(scale):
    c = dict(workloads.RECOMBINATION)
    c["beta_ep"] *= scale
    c["beta_np"] *= scale
    return c


def test_full_steps_conserve_charge_with_recombination(orc):
    """Avalanche steps with (strongly scaled) recombination: the charge identity
    sum(n+ - n_e - n-) = initial + outflow holds exactly and both recombinations fire."""
    cfg = _cfg(coeffs=_recomb_coeffs(1e7), seed_n0=3000, steps=40)
    sim = orc.Sim(cfg)
    sim.seed_gaussian(cfg["seed_n0"], cfg["seed_centre"], cfg["seed_sigma"])
    d0 = sim.diagnostics()
    sim.step(cfg["dt"], 40)
    d = sim.diagnostics()
    assert d["charge"] == d0["charge"] + d["outflow_weight"]
    assert d["n_plus"] - d["n_minus"] - d["weight"] == d["charge"]
    assert d["fires"][3] > 0 and d["fires"][4] > 0


def test_ion_only_cells_react(orc):
    """A cell holding ions of both signs and no electrons still takes its KMC step
    (ion-ion recombination is the only reaction that can fire there)."""
    cfg = _cfg(coeffs=_recomb_coeffs(1e9))
    sim = orc.Sim(cfg)
    nc = 32 ** 3
    plus = np.zeros(nc, dtype=np.int64)
    minus = np.zeros(nc, dtype=np.int64)
    plus[:500] = 40
    minus[:500] = 30
    sim.set_counts("plus", plus)
    sim.set_counts("minus", minus)
    sim.step(cfg["dt"], 1)
    p1, m1 = sim.counts("plus"), sim.counts("minus")
    fired = 30 - m1[:500]
    assert np.array_equal(40 - p1[:500], fired) and fired.sum() > 0
    assert sim.diagnostics()["fires"][4] == fired.sum()
    assert p1[500:].sum() == 0 and m1[500:].sum() == 0
    # without recombination nothing happens there
    sim0 = orc.Sim(_cfg())
    sim0.set_counts("plus", plus)
    sim0.set_counts("minus", minus)
    sim0.step(cfg["dt"], 1)
    assert np.array_equal(sim0.counts("minus"), minus)
