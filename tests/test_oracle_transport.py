"""Pins of the oracle's particle transport and particle-mesh transfers: ensemble
averages of the Ito kernel (drift v dt, diffusive variance 2 D dt per axis), the
electron drift sign, removal at the domain faces, NGP totals, CIC weights and
conservation, and exact interpolation of linear fields."""
import math

import numpy as np
import pytest

from paper_2307_01797_amd import workloads


def test_drift_and_diffusion_ensemble_averages(orc):
    """Reactions off, 64^3 grid so that no particle leaves: after 200 steps of 1 ps the
    mean displacement is -mu E t along z and the per-axis variance is 2 D t."""
    cfg = workloads.preset("avalanche_32", grid=(64, 64, 64),
                           coeffs=dict(alpha_A=0.0, eta=0.0))
    sim = orc.Sim(cfg)
    sim.seed_gaussian(10000, (320e-6, 320e-6, 320e-6), 50e-6)
    xi0, w0, id0 = sim.particles()
    sim.step(1e-12, 200)
    xi1, w1, id1 = sim.particles()
    assert np.array_equal(np.sort(id0), np.sort(id1))  # nothing created or lost
    o0, o1 = np.argsort(id0), np.argsort(id1)
    disp = (xi1[o1] - xi0[o0]) * cfg["dx"]
    t = 200e-12
    mu = orc.mobility(cfg, 1e7)
    n = disp.shape[0]
    sd = math.sqrt(2 * 0.1 * t)
    assert sd == pytest.approx(6.325e-6, rel=1e-3)
    mean_z = -mu * 1e7 * t
    assert mean_z == pytest.approx(-41.84e-6, rel=1e-3)
    assert abs(disp[:, 2].mean() - mean_z) < 5 * sd / math.sqrt(n)
    for a in (0, 1):
        assert abs(disp[:, a].mean()) < 5 * sd / math.sqrt(n)
    for a in range(3):
        v = disp[:, a].var()
        assert abs(v / sd**2 - 1) < 5 * math.sqrt(2.0 / n)


def test_outflow_and_ngp_totals(orc):
    cfg = workloads.preset("avalanche_32", coeffs=dict(alpha_A=0.0, eta=0.0),
                           E=(0.0, 0.0, 2.0e8))  # strong field: particles leave at z = 0
    sim = orc.Sim(cfg)
    sim.seed_gaussian(5000, (160e-6, 160e-6, 160e-6), 50e-6)
    d0 = sim.diagnostics()
    n0 = d0["n_particles"]
    assert n0 < 5000  # draws outside the box were discarded
    sim.step(1e-12, 30)
    d1 = sim.diagnostics()
    assert d1["outflow_weight"] > 0
    assert d1["weight"] + d1["outflow_weight"] == n0
    xi, w, ids = sim.particles()
    assert np.all(xi >= 0) and np.all(xi < 32)
    ngp = sim.ngp_weight()
    assert ngp.sum() == w.sum()
    # NGP equals a histogram of floor(xi)
    c = np.floor(xi).astype(np.int64)
    lin = c[:, 0] + 32 * (c[:, 1] + 32 * c[:, 2])
    assert np.array_equal(np.bincount(lin, weights=w.astype(float), minlength=32**3).astype(np.int64), ngp)


def test_cic_single_particle_weights(orc):
    cfg = workloads.preset("avalanche_32", grid=(8, 8, 8))
    xi = np.array([[3.75, 4.5, 2.125]])
    g = orc.cic_deposit(cfg, xi, np.array([1.0])).reshape(8, 8, 8)  # [k, j, i]
    # tent weights about cell centres (i + 1/2): x -> nodes 3,4 with 0.75, 0.25
    fx = {3: 0.75, 4: 0.25}
    fy = {4: 1.0, 5: 0.0}
    fz = {1: 0.375, 2: 0.625}
    exp = np.zeros((8, 8, 8))
    for i, a in fx.items():
        for j, b in fy.items():
            for k, c in fz.items():
                exp[k, j, i] += a * b * c
    assert np.allclose(g, exp, atol=1e-15)
    assert g.sum() == pytest.approx(1.0, abs=1e-15)


def test_cic_wall_folding_conserves(orc):
    cfg = workloads.preset("avalanche_32", grid=(8, 8, 8))
    rng = np.random.default_rng(3)
    xi = rng.random((2000, 3)) * 8
    xi[:100, 0] = rng.random(100) * 0.5          # outer half of the wall cells
    xi[100:200, 2] = 8 - rng.random(100) * 0.5
    q = rng.random(2000)
    g = orc.cic_deposit(cfg, xi, q)
    assert g.sum() == pytest.approx(q.sum(), rel=1e-13)
    assert g.min() >= 0.0


def test_cic_interpolates_linear_fields_exactly(orc):
    cfg = workloads.preset("avalanche_32", grid=(8, 8, 8))
    k, j, i = np.meshgrid(np.arange(8), np.arange(8), np.arange(8), indexing="ij")
    f = (2.0 * (i + 0.5) - 3.0 * (j + 0.5) + 0.5 * (k + 0.5) + 1.0).ravel()
    rng = np.random.default_rng(4)
    xi = 0.5 + rng.random((500, 3)) * 7.0       # between the outermost cell centres
    v = orc.cic_interp(cfg, f, xi)
    exact = 2.0 * xi[:, 0] - 3.0 * xi[:, 1] + 0.5 * xi[:, 2] + 1.0
    assert np.allclose(v, exact, atol=1e-12)
