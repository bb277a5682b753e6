"""Pins of the oracle's random-number layer (counter-based Philox4x32-10, Box-Muller
normals, Poisson deviates) against statistics fixed by their definitions."""
import numpy as np
import pytest
from scipy import stats


def _words(orc, n, tag=1, key=(1, 0)):
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(n, dtype=np.uint32)
    ctr[:, 3] = tag << 24
    return orc.philox_many(ctr, key)


def test_philox_bit_balance(orc):
    w = _words(orc, 1 << 15).ravel()
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.float64)
    frac = bits.mean(axis=0)
    se = 0.5 / np.sqrt(w.size)
    assert np.all(np.abs(frac - 0.5) < 5 * se)


def test_philox_byte_uniformity(orc):
    w = _words(orc, 1 << 15, tag=3)
    b = w.view(np.uint8).ravel()
    hist = np.bincount(b, minlength=256)
    chi2, p = stats.chisquare(hist)
    assert p > 1e-4


def test_philox_avalanche_and_key(orc):
    rng = np.random.default_rng(7)
    dist = []
    for _ in range(400):
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64).astype(np.uint32)
        bit = rng.integers(0, 128)
        ctr2 = ctr.copy()
        ctr2[bit // 32] ^= np.uint32(1 << (bit % 32))
        a = orc.philox(ctr, (5, 9))
        b = orc.philox(ctr2, (5, 9))
        dist.append(sum(bin(int(x) ^ int(y)).count("1") for x, y in zip(a, b)))
    d = np.asarray(dist, dtype=float)
    assert abs(d.mean() - 64.0) < 5 * 4.0 / np.sqrt(d.size)
    # a different key gives a different block
    assert not np.array_equal(orc.philox([1, 2, 3, 4], (1, 0)), orc.philox([1, 2, 3, 4], (1, 1)))
    # determinism
    assert np.array_equal(orc.philox([1, 2, 3, 4], (1, 0)), orc.philox([1, 2, 3, 4], (1, 0)))


def test_normals_standard_normal(orc):
    n = 30000
    z = np.array([orc.normals3(i * 977 + 5, 3, 1, 0) for i in range(n)])
    for a in range(3):
        assert abs(z[:, a].mean()) < 5 / np.sqrt(n)
        assert abs(z[:, a].var() - 1.0) < 5 * np.sqrt(2.0 / n)
        assert stats.kstest(z[:, a], "norm").pvalue > 1e-4
    c = np.corrcoef(z.T)
    assert np.all(np.abs(c[np.triu_indices(3, 1)]) < 5 / np.sqrt(n))
    # a different step gives independent normals for the same particle
    z2 = np.array([orc.normals3(i * 977 + 5, 4, 1, 0) for i in range(2000)])
    assert abs(np.corrcoef(z[:2000, 2], z2[:, 2])[0, 1]) < 5 / np.sqrt(2000)


@pytest.mark.parametrize("lam", [0.3, 4.0, 9.5, 10.0, 37.5, 1000.0])
def test_poisson_sampler(orc, lam):
    n = 20000
    draws = np.array([orc.poisson_draw(lam, c, 11)[0] for c in range(n)])
    assert draws.min() >= 0
    assert abs(draws.mean() - lam) < 5 * np.sqrt(lam / n)
    assert abs(draws.var() - lam) < 6 * lam * np.sqrt(2.0 / n) + 5 * np.sqrt(lam / n)
    # goodness of fit against the Poisson pmf, tail bins merged
    lo, hi = int(stats.poisson.ppf(1e-4, lam)), int(stats.poisson.ppf(1 - 1e-4, lam))
    edges = np.arange(lo, hi + 2)
    obs = np.array([np.sum(draws < lo)] + [np.sum(draws == k) for k in range(lo, hi + 1)] +
                   [np.sum(draws > hi)])
    exp = n * np.array([stats.poisson.cdf(lo - 1, lam)] + [stats.poisson.pmf(k, lam) for k in range(lo, hi + 1)] +
                       [stats.poisson.sf(hi, lam)])
    # merge bins with small expectation
    o2, e2, acc_o, acc_e = [], [], 0, 0.0
    for o, e in zip(obs, exp):
        acc_o += o; acc_e += e
        if acc_e >= 20:
            o2.append(acc_o); e2.append(acc_e); acc_o, acc_e = 0, 0.0
    if acc_e > 0:
        o2[-1] += acc_o; e2[-1] += acc_e
    e2 = np.asarray(e2) * (n / np.sum(e2))
    assert stats.chisquare(o2, e2).pvalue > 1e-4


def test_poisson_draw_accounting(orc):
    # inversion uses exactly one uniform; lambda = 0 uses none
    assert orc.poisson_draw(0.0, 1, 1) == (0, 0)
    assert orc.poisson_draw(2.0, 1, 1)[1] == 1
    # PTRS uses two uniforms per trial
    assert orc.poisson_draw(50.0, 1, 1)[1] % 2 == 0
