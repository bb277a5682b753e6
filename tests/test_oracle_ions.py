"""Pins of the oracle's mobile ions (the lattice jump process of move_ions in
oracle/sim.c: per-cell integer ion counts drifting with q mu_ion E and diffusing with
D_ion, first-order upwind rates, Poisson counts per face and step, capped at the ions
left).  Each pin is a law the mathematics fixes:
  - drift: a cloud of positive ions in a uniform field moves by mu_ion E t on average,
    negative ions by -mu_ion E t, with the spread of independent Bernoulli hops;
  - diffusion: with no field the variance per axis grows as 2 D_ion t / dx^2;
  - conservation: counts stay non-negative and ions only leave through the domain
    faces (tallied), also when the per-step hop probabilities are large;
  - the self-consistent field: a charged sheet of ions in a plane gap drifts with the
    face fields of the exact one-dimensional solution, (3 E_a + E_b)/4 and
    (E_a + 3 E_b)/4 on its two faces;
  - the charge identity of full steps with ions moving."""
import numpy as np
import pytest

from paper_2307_01797_amd import workloads

E_CHARGE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def _uniform(E, mu_ion, D_ion, grid=(16, 16, 48)):
    cfg = workloads.preset("avalanche_32", grid=grid, E=(0.0, 0.0, E))
    cfg["coeffs"].update(mu_ion=mu_ion, D_ion=D_ion)
    return cfg


def _cloud(orc, cfg, cell_ijk, n_plus, n_minus):
    sim = orc.Sim(cfg)
    nx, ny, nz = cfg["grid"]
    c = cell_ijk[0] + nx * (cell_ijk[1] + ny * cell_ijk[2])
    p = np.zeros(nx * ny * nz, dtype=np.int64)
    m = np.zeros_like(p)
    p[c] = n_plus
    m[c] = n_minus
    sim.set_counts("plus", p)
    sim.set_counts("minus", m)
    return sim


def _moments(counts, grid, axis):
    nx, ny, nz = grid
    ijk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    coord = np.stack([a.transpose(2, 1, 0).ravel() for a in ijk])[axis]
    n = counts.sum()
    mean = (counts * coord).sum() / n
    var = (counts * (coord - mean) ** 2).sum() / n
    return n, mean, var


def test_drift_of_positive_and_negative_ions(orc):
    E, mu, dt, K = 1e7, 2e-4, 1e-10, 20
    cfg = _uniform(E, mu, 0.0)
    N = 1_000_000
    k0 = 24
    sim = _cloud(orc, cfg, (8, 8, k0), N, N)
    for _ in range(K):
        sim.step(dt)        # transport, then the step counter (keys the next draws)
    p = mu * E * dt / cfg["dx"]          # hop probability per step (0.02)
    for which, sign in (("plus", 1.0), ("minus", -1.0)):
        n, mean, var = _moments(sim.counts(which), cfg["grid"], 2)
        assert n == N
        disp = mean - k0
        sd = np.sqrt(K * p / N)
        assert abs(disp - sign * K * p) < 5 * sd, (which, disp)
        assert var == pytest.approx(K * p * (1 - p), rel=0.02)
        for ax in (0, 1):
            assert _moments(sim.counts(which), cfg["grid"], ax)[2] == 0.0
        # upwind drift without diffusion: no ion ever moves against its force
        col = sim.counts(which).reshape(cfg["grid"][2], -1).sum(axis=1)
        behind = col[:k0] if sign > 0 else col[k0 + 1:]
        assert behind.sum() == 0


def test_diffusion_law(orc):
    D, dt, K = 1e-6, 1e-6, 25
    cfg = _uniform(0.0, 0.0, D, grid=(24, 24, 24))
    N = 1_000_000
    sim = _cloud(orc, cfg, (12, 12, 12), N, 0)
    for _ in range(K):
        sim.step(dt)        # transport, then the step counter (keys the next draws)
    want = 2 * D * K * dt / cfg["dx"] ** 2   # 0.5 cells^2
    vs = []
    for ax in range(3):
        n, mean, var = _moments(sim.counts("plus"), cfg["grid"], ax)
        assert n == N
        assert abs(mean - 12) < 5 * np.sqrt(want / N)
        vs.append(var)
    # the spread of one axis scatters by about 0.26% between seeds
    assert np.all(np.abs(np.array(vs) / want - 1) < 0.015)
    assert sim.counts("minus").sum() == 0


def test_conservation_with_large_hops_and_outflow(orc):
    # hop probabilities of order one per face: the caps bind, counts stay >= 0, and
    # every ion is either inside or tallied as outflow
    cfg = _uniform(3e7, 2e-4, 2e-5, grid=(6, 5, 7))
    rng = np.random.default_rng(3)
    n = cfg["grid"][0] * cfg["grid"][1] * cfg["grid"][2]
    p = rng.integers(0, 50, n)
    m = rng.integers(0, 50, n)
    sim = orc.Sim(cfg)
    sim.set_counts("plus", p)
    sim.set_counts("minus", m)
    for _ in range(10):
        sim.step(2e-9)
        cp, cm = sim.counts("plus"), sim.counts("minus")
        assert cp.min() >= 0 and cm.min() >= 0
        d = sim.diagnostics()
        assert cp.sum() + d["ion_outflow_plus"] == p.sum()
        assert cm.sum() + d["ion_outflow_minus"] == m.sum()
    assert d["ion_outflow_plus"] > 0 and d["ion_outflow_minus"] > 0


def test_immobile_by_default(orc):
    cfg = workloads.preset("avalanche_32")
    sim = orc.Sim(cfg)
    p = np.arange(32 ** 3, dtype=np.int64) % 7
    sim.set_counts("plus", p)
    sim.transport(1e-9)
    assert np.array_equal(sim.counts("plus"), p)


def test_sheet_drifts_with_its_own_field(orc):
    """A sheet of N positive ions in plane k0 of a plane gap, no electrons.  The solved
    field is linear on each side: E_a above and E_b below with E_a - E_b = sigma / eps0
    and E_b z0 + E_a (L - z0) = -V (z0 the sheet's centre), the sheet's own cell at
    (E_a + E_b) / 2; the ions hop with the face means (3 E_a + E_b) / 4 up and
    (E_a + 3 E_b) / 4 down."""
    nx, ny, nz, L, V = 4, 4, 32, 1e-3, 2e3
    dx = L / nz
    mu, dt = 2e-4, 2e-9
    cfg = workloads.preset("streamer_64", grid=(nx, ny, nz), dx=dx, V_anode=V, n_ppc=0)
    cfg["coeffs"].update(mu_ion=mu, D_ion=0.0)
    per_cell = 2_000_000      # the sheet's own field dominates V / L: it spreads both ways
    k0 = 12
    sim = orc.Sim(cfg)
    p = np.zeros(nx * ny * nz, dtype=np.int64)
    p[k0 * nx * ny:(k0 + 1) * nx * ny] = per_cell
    sim.set_counts("plus", p)
    sim.transport(dt)
    sigma = E_CHARGE * per_cell / dx ** 2          # surface charge of the sheet
    z0 = (k0 + 0.5) * dx
    Eb = (-V - sigma / EPS0 * (L - z0)) / L
    Ea = Eb + sigma / EPS0
    Ez = sim.field()[3].reshape(nz, ny, nx)[:, 0, 0]
    assert Ez[k0 - 3] == pytest.approx(Eb, rel=1e-9)
    assert Ez[k0 + 3] == pytest.approx(Ea, rel=1e-9)
    assert Ez[k0] == pytest.approx(0.5 * (Ea + Eb), rel=1e-9)
    up = max(0.0, mu * (3 * Ea + Eb) / 4) * dt / dx
    down = max(0.0, -mu * (Ea + 3 * Eb) / 4) * dt / dx
    assert up > 0.01 and down > 0.01          # the sheet spreads both ways
    cnt = sim.counts("plus").reshape(nz, ny * nx).sum(axis=1)
    Ntot = per_cell * nx * ny
    assert cnt.sum() == Ntot
    for k, want in ((k0 + 1, up), (k0 - 1, down)):
        assert cnt[k] / Ntot == pytest.approx(want, abs=5 * np.sqrt(want / Ntot))


def test_charge_identity_with_moving_ions(orc):
    cfg = workloads.preset("avalanche_32", E=(0.0, 0.0, 1.5e7))
    cfg["coeffs"].update(mu_ion=3e-2, D_ion=5e-3)   # exaggerated: ions reach the faces
    sim = orc.Sim(cfg)
    sim.seed_gaussian(cfg["seed_n0"], cfg["seed_centre"], cfg["seed_sigma"])
    q0 = sim.diagnostics()["charge"]
    sim.step(cfg["dt"], 60)
    d = sim.diagnostics()
    assert d["ion_outflow_plus"] > 0
    assert d["charge"] == q0 + d["outflow_weight"] - d["ion_outflow_plus"] + d["ion_outflow_minus"]
    assert min(sim.counts("plus").min(), sim.counts("minus").min()) >= 0


def test_small_mean_faces_are_independent_poisson(orc):
    """Cells with a small total mean draw the number of movers and then split it over
    the faces: each face's count must still be Poisson(lambda_f), independent of the
    others.  Isolated source cells (two empty cells between sources) let every face's
    count be read from the receiving neighbour after one step."""
    E, mu, D, dt = 1e7, 2e-4, 1e-2, 1e-10     # means 0.6 per diffusion face, 1.8 up
    cfg = _uniform(E, mu, D, grid=(36, 36, 9))
    nx, ny, nz = cfg["grid"]
    n0 = 60
    src = [(i, j, 4) for i in range(1, nx - 1, 3) for j in range(1, ny - 1, 3)]
    p = np.zeros(nx * ny * nz, dtype=np.int64)
    for (i, j, k) in src:
        p[i + nx * (j + ny * k)] = n0
    sim = orc.Sim(cfg)
    sim.set_counts("plus", p)
    sim.step(dt)
    c = sim.counts("plus").reshape(nz, ny, nx)
    K = np.array([[c[k, j, i - 1], c[k, j, i + 1], c[k, j - 1, i], c[k, j + 1, i], c[k - 1, j, i],
                   c[k + 1, j, i]] for (i, j, k) in src], dtype=float)
    r_d = D / cfg["dx"] ** 2
    r_up = mu * E / cfg["dx"] + r_d
    lam = n0 * dt * np.array([r_d, r_d, r_d, r_d, r_d, r_up])
    assert lam.sum() < 10.0                     # the split way
    m = len(src)
    for f in range(6):
        assert K[:, f].mean() == pytest.approx(lam[f], abs=5 * np.sqrt(lam[f] / m))
        assert K[:, f].var() == pytest.approx(lam[f], rel=5 * np.sqrt(2.0 / m) + 0.05)
    cov = np.cov(K.T)
    off = cov[~np.eye(6, dtype=bool)]
    assert np.abs(off).max() < 5 * np.sqrt(lam.max() * lam.max() / m)
    # a multinomial split of a fixed total would make the faces anticorrelated
    assert abs(np.corrcoef(K[:, 4], K[:, 5])[0, 1]) < 5 / np.sqrt(m)
