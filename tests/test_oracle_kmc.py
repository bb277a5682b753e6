"""Pins of the oracle's per-cell KMC against closed forms: transport/rate coefficients
at the avalanche field, Poisson one-leap counts, the linear birth-death process
(extinction probability and mean growth), the discrete tau-leap growth law, a pure
death process (exact binomial law, exercises the critical-reaction branch), and the
invariants (charge, non-negativity)."""
import math

import numpy as np
import pytest
from scipy import stats

from paper_2307_01797_amd import workloads

DT = 1e-12


def _cfg(**kw):
    return workloads.preset("avalanche_32", **kw)


def test_rates_at_avalanche_field(orc):
    cfg = _cfg()
    mu = orc.mobility(cfg, 1e7)
    k = orc.rates(cfg, 1e7)
    # derived values of the synthetic air coefficients at 10 MV/m
    assert mu == pytest.approx(0.020919, rel=1e-4)
    assert k[0] == pytest.approx(1.3419e10, rel=1e-4)
    assert k[1] == pytest.approx(4.1838e8, rel=1e-4)
    assert k[2] == 0.0
    # photo-emission ratio
    k2 = orc.rates(workloads.preset("streamer_64"), 1e7)
    assert k2[2] == pytest.approx(0.06 * k2[0], rel=1e-12)
    # alpha(0) = 0: no ionization without field
    assert orc.rates(cfg, 0.0)[0] == 0.0


def _run_cells(orc, cfg, X0, nsteps, n, E=1e7, k=None):
    X = np.zeros((n, 4), dtype=np.int64)
    X[:, 0] = X0
    if k is None:
        k = orc.rates(cfg, E)
    K = np.tile(k, (n, 1))
    F = np.zeros((n, 5), dtype=np.int64)
    for s in range(nsteps):
        X, f = orc.kmc_cells(cfg, X, K, DT, s)
        F += f
        assert X.min() >= 0
        # every reaction conserves charge: -e + M+ - M- is invariant
        assert np.all(-X[:, 0] + X[:, 1] - X[:, 2] == -X0)
    return X, F


def test_pure_tau_one_leap_counts(orc):
    cfg = _cfg(kmc="pure_tau")
    n = 40000
    X, F = _run_cells(orc, cfg, 200, 1, n)
    k = orc.rates(cfg, 1e7)
    for r, lam in ((0, 200 * k[0] * DT), (1, 200 * k[1] * DT)):
        assert lam == pytest.approx([2.684, 0.0837][r], rel=2e-3)
        obs = np.bincount(F[:, r])
        kmax = len(obs) - 1
        exp = n * stats.poisson.pmf(np.arange(kmax + 1), lam)
        exp[-1] += n * stats.poisson.sf(kmax, lam)
        keep = exp >= 10
        o = np.append(obs[keep], obs[~keep].sum())
        e = np.append(exp[keep], exp[~keep].sum())
        if e[-1] == 0:
            o, e = o[:-1], e[:-1]
        e = e * o.sum() / e.sum()
        assert stats.chisquare(o, e).pvalue > 1e-4


def test_birth_death_extinction_and_mean(orc):
    """One electron at 10 MV/m for 50 ps: linear birth-death process."""
    cfg = _cfg()
    n, K = 60000, 50
    X, F = _run_cells(orc, cfg, 1, K, n)
    k = orc.rates(cfg, 1e7)
    lam, mu, t = k[0], k[1], K * DT
    r = lam - mu
    p0 = mu * (math.exp(r * t) - 1) / (lam * math.exp(r * t) - mu)
    assert p0 == pytest.approx(0.01514, rel=2e-3)
    frac = np.mean(X[:, 0] == 0)
    assert abs(frac - p0) < 5 * math.sqrt(p0 * (1 - p0) / n)
    mean = math.exp(r * t)
    var = (lam + mu) / r * math.exp(r * t) * (math.exp(r * t) - 1)
    assert abs(X[:, 0].mean() - mean) < 5 * math.sqrt(var / n)
    # selection probability of ionization among electron-consuming/producing events
    pr = lam / (lam + mu)
    tot = F[:, 0] + F[:, 1]
    assert abs(F[:, 0].sum() / tot.sum() - pr) < 5 * math.sqrt(pr * (1 - pr) / tot.sum())


def test_mean_growth_continuous_vs_discrete(orc):
    """Hybrid in its SSA regime follows exp((k_a - k_e) t); pure tau-leaping and the
    hybrid's leap regime follow the discrete law (1 + (k_a - k_e) dt)^K."""
    K = 50
    k = orc.rates(_cfg(), 1e7)
    r = k[0] - k[1]
    cont = math.exp(r * K * DT)
    disc = (1 + r * DT) ** K
    assert cont / disc - 1 > 3e-3  # the two laws are distinguishable

    def check(X0, n, cfg, target, other):
        X, _ = _run_cells(orc, cfg, X0, K, n)
        m = X[:, 0].mean() / X0
        var1 = (k[0] + k[1]) / r * cont * (cont - 1)       # per initial electron
        se = math.sqrt(var1 / X0 / n)
        assert abs(m - target) < 5 * se, (m, target, se)
        assert abs(m - other) > 3 * se

    check(20, 40000, _cfg(kmc="pure_tau"), disc, cont)
    check(20, 40000, _cfg(), cont, disc)          # SSA exception (A dt <= 1)
    check(1000, 6000, _cfg(), disc, cont)         # leap branch (A dt > 1)


def test_pure_death_is_binomial(orc):
    """With ionization off and strong attachment, a cell of 3 electrons is always in the
    critical regime (X_e < N_c) and the hybrid must reproduce the exact death process:
    X_e(dt) ~ Binomial(3, exp(-k_eta dt))."""
    cfg = _cfg()
    n = 40000
    keta = 2.0e12
    k = np.array([0.0, keta, 0.0])
    X, F = _run_cells(orc, cfg, 3, 1, n, k=k)
    p = math.exp(-keta * DT)
    obs = np.bincount(X[:, 0], minlength=4)
    exp = n * stats.binom.pmf(np.arange(4), 3, p)
    assert stats.chisquare(obs, exp).pvalue > 1e-4
    # a large, strongly attaching cell is leapt: with eps = inf (any leap accepted) the
    # rejection path must keep populations non-negative; with a small eps the leap
    # bound of step 4 must bring the mean to the exact value 100 exp(-k_eta dt)
    X2, _ = _run_cells(orc, cfg, 100, 1, 4000, k=k)
    assert X2.min() >= 0
    X3, _ = _run_cells(orc, _cfg(kmc_eps=0.02), 100, 1, 4000, k=k)
    assert X3.min() >= 0
    assert abs(X3[:, 0].mean() - 100 * p) < 0.03 * 100 * p
    assert abs(X2[:, 0].mean() - 100 * p) > 0.3 * 100 * p  # eps = inf is visibly coarser


def test_kmc_stream_determinism(orc):
    cfg = _cfg()
    X = np.zeros((100, 4), dtype=np.int64)
    X[:, 0] = np.arange(100) * 7
    K = np.tile(orc.rates(cfg, 1e7), (100, 1))
    a = orc.kmc_cells(cfg, X, K, DT, 5)
    b = orc.kmc_cells(cfg, X, K, DT, 5)
    c = orc.kmc_cells(cfg, X, K, DT, 6)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(a[1], c[1])
