"""Pins of the oracle's quadratic B-spline (TSC) particle shape, the higher-order
deposition of the paper's future-work section, used for the field coupling (conductivity
and charge deposits, field interpolation) when a workload selects shape "tsc".  The pins
come from the mathematics of the shape, not from its formula:
  - moments: the weights sum to one and reproduce x and x^2 + 1/4 inside the grid;
  - the shape is the CIC tent averaged over a unit box (the CIC deposit integrated
    numerically over the box);
  - continuity of every weight as the particle crosses a cell face;
  - wall folding keeps the total and a convex combination, also for points outside;
  - interpolation is the transpose of deposition (same weights), exact for linear
    fields inside the grid;
  - a neutral plasma of electrons and ions on the same cell centres has zero charge
    (ions take the particles' shape);
  - a one-dimensional closed form of the semi-implicit step: a plane layer of
    conductive plasma whose TSC-smoothed conductivity profile splits the gap voltage
    like resistors in series, and electrons that move with the TSC average of E^{k+1}."""
import numpy as np
import pytest

from paper_2307_01797_amd import workloads

from tsc_layer_case import make_layer


def _line(n=16, shape="tsc"):
    # one-dimensional grid along x (ny = nz = 1: the other axes take all the weight)
    return workloads.preset("streamer_64", grid=(n, 1, 1), dx=1e-5, shape=shape)


def _box(shape="tsc", grid=(12, 10, 14)):
    return workloads.preset("streamer_64", grid=grid, dx=1e-5, shape=shape)


def test_moments_inside_the_grid(orc):
    cfg = _box()
    nx, ny, nz = cfg["grid"]
    rng = np.random.default_rng(5)
    lo = np.array([1.5, 1.5, 1.5])
    hi = np.array([nx, ny, nz]) - 1.5
    xi = lo + (hi - lo) * rng.random((200, 3))
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    centres = [i.ravel() + 0.5, j.ravel() + 0.5, k.ravel() + 0.5]
    for p in xi:
        g = orc.tsc_deposit(cfg, p[None, :], np.ones(1))
        assert g.min() >= 0.0
        assert g.sum() == pytest.approx(1.0, abs=1e-14)
        for a in range(3):
            assert (g * centres[a]).sum() == pytest.approx(p[a], abs=1e-12)
            assert (g * centres[a] ** 2).sum() == pytest.approx(p[a] ** 2 + 0.25, abs=1e-11)
        assert np.count_nonzero(g) <= 27


def test_tsc_is_the_box_average_of_cic(orc):
    n = 16
    tsc, cic = _line(n, "tsc"), _line(n, "cic")
    rng = np.random.default_rng(6)
    m = 20000
    for x in 2.0 + (n - 4.0) * rng.random(12):
        w_tsc = orc.tsc_deposit(tsc, np.array([[x, 0.5, 0.5]]), np.ones(1))
        y = x - 0.5 + (np.arange(m) + 0.5) / m         # midpoints of a unit box about x
        pts = np.stack([y, np.full(m, 0.5), np.full(m, 0.5)], axis=1)
        w_box = orc.cic_deposit(cic, pts, np.full(m, 1.0 / m))
        assert np.abs(w_tsc - w_box).max() < 1e-7, x


def test_weights_continuous_across_faces(orc):
    cfg = _line(16)
    for face in (3.0, 7.0, 11.0):
        for eps in (1e-6, 1e-9):
            a = orc.tsc_deposit(cfg, np.array([[face - eps, 0.5, 0.5]]), np.ones(1))
            b = orc.tsc_deposit(cfg, np.array([[face + eps, 0.5, 0.5]]), np.ones(1))
            assert np.abs(a - b).max() < 4 * eps


def test_walls_fold_and_conserve(orc):
    cfg = _box(grid=(6, 5, 7))
    rng = np.random.default_rng(7)
    # points near and beyond every wall (diffusive positions can leave the grid)
    xi = rng.uniform(-1.5, 1.0, size=(300, 3)) * rng.choice([1, -1], size=(300, 3))
    xi = np.where(xi < 0, xi, np.array(cfg["grid"]) - xi)
    q = rng.uniform(0.5, 2.0, 300)
    g = orc.tsc_deposit(cfg, xi, q)
    assert g.min() >= 0.0
    assert g.sum() == pytest.approx(q.sum(), rel=1e-13)
    # a point at the centre of a wall cell keeps 7/8 along that axis (3/4 own + 1/8 folded)
    c = orc.tsc_deposit(_line(8), np.array([[0.5, 0.5, 0.5]]), np.ones(1))
    assert c[0] == 0.875 and c[1] == 0.125 and c[2:].sum() == 0.0


def test_interpolation_is_the_transpose_and_exact_for_linear_fields(orc):
    cfg = _box()
    nx, ny, nz = cfg["grid"]
    rng = np.random.default_rng(8)
    F = rng.normal(size=nx * ny * nz)
    xi = rng.uniform(0.0, 1.0, size=(50, 3)) * np.array(cfg["grid"])
    v = orc.tsc_interp(cfg, F, xi)
    for p, vp in zip(xi, v):
        g = orc.tsc_deposit(cfg, p[None, :], np.ones(1))
        assert (g * F).sum() == pytest.approx(vp, rel=1e-12, abs=1e-12)
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    lin = 3.0 + 0.7 * (i.ravel() + 0.5) - 1.3 * (j.ravel() + 0.5) + 0.2 * (k.ravel() + 0.5)
    inner = 1.5 + rng.random((100, 3)) * (np.array(cfg["grid"]) - 3.0)
    got = orc.tsc_interp(cfg, lin, inner)
    want = 3.0 + 0.7 * inner[:, 0] - 1.3 * inner[:, 1] + 0.2 * inner[:, 2]
    assert np.abs(got - want).max() < 1e-12


def _plasma_layer(orc, shape):
    c = make_layer(workloads.preset("streamer_64"), shape)
    sim = orc.Sim(c["cfg"])
    sim.set_particles(c["xi"], c["w"], c["ids"])
    sim.set_counts("plus", c["nplus"])
    return sim, c["cfg"], c


def test_neutral_layer_has_no_charge(orc):
    sim, cfg, _ = _plasma_layer(orc, "tsc")
    assert np.abs(sim.charge_density()).max() == 0.0
    # the CIC shape deposits a centre's charge in its own cell: also neutral
    sim, cfg, _ = _plasma_layer(orc, "cic")
    assert np.abs(sim.charge_density()).max() == 0.0


def test_layer_closed_form_with_tsc(orc):
    sim, cfg, c = _plasma_layer(orc, "tsc")
    nx, ny, nz = cfg["grid"]
    sim.transport(cfg["dt"])
    phi, Ex, Ey, Ez = sim.field()
    Ez1 = c["Ez_col"]
    col = Ez.reshape(nz, ny, nx)
    assert np.abs(col - Ez1[:, None, None]).max() < 1e-9 * np.abs(Ez1).max()
    assert np.abs(Ex).max() < 1e-9 * np.abs(Ez1).max()
    # each electron (on a centre) moves with the TSC average of E^{k+1} along z
    xi, w, ids = sim.particles()
    o = np.argsort(ids)
    p = np.argsort(c["ids"])
    d = xi[o] - c["xi"][p]
    assert np.allclose(d[:, 2], c["dz"][p], rtol=1e-9, atol=0)
    assert np.abs(d[:, :2]).max() < 1e-12
    # the smoothed profile really differs from the CIC one (which has a sharp edge)
    sim2, cfg2, _ = _plasma_layer(orc, "cic")
    sim2.transport(cfg["dt"])
    assert np.abs(sim2.field()[3].reshape(nz, ny, nx)[:, 0, 0] - Ez1).max() > 1e-3 * np.abs(Ez1).max()
