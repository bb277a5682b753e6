"""Pins of the oracle's dynamic time-step rule (the paper's closing remark on its final
algorithm names CFL- or physics-based stepping as the next step; the rule's reading is
stated in oracle/sim.c).  Each pin checks what a limit promises through the rest of the
method, not by retyping its formula:
  - drift limit: in a uniform field with D = 0, one transport moves every electron by
    exactly c_drift cells against the field;
  - diffusion limit: with the field negligible, the per-axis spread of one transport
    has variance c_diff (cells^2);
  - ionization limit: the reaction step's mean ionizations per electron equal c_ion;
  - the field bound: a plane vacuum gap gives Emax = V / L; every particle's
    interpolated field stays below Emax;
  - asking for the step first changes nothing in the step itself (the initial field
    the query computes is the one the first transport would compute)."""
import numpy as np
import pytest

from paper_2307_01797_amd import workloads


def _uniform(E=1e7, **kw):
    cfg = workloads.preset("avalanche_32", E=(0.0, 0.0, E), **kw)
    return cfg


def _seeded(orc, cfg):
    sim = orc.Sim(cfg)
    sim.seed_gaussian(cfg["seed_n0"], cfg["seed_centre"], cfg["seed_sigma"])
    return sim


def test_drift_limit_moves_every_electron_c_drift_cells(orc):
    for E, c in ((1e7, 0.5), (3e6, 0.25), (1e5, 0.8)):
        cfg = _uniform(E, coeffs=dict(D=0.0))
        sim = _seeded(orc, cfg)
        dt, Em = sim.stable_dt({"dt_max": 1.0, "c_drift": c})
        assert Em == E
        xi0, w0, id0 = sim.particles()
        sim.transport(dt)
        xi1, w1, id1 = sim.particles()
        # electrons that crossed a face are removed: compare the others by id
        o = np.argsort(id0)
        j = o[np.searchsorted(id0, id1, sorter=o)]
        assert np.array_equal(id0[j], id1) and len(id1) > 0.99 * len(id0)
        d = xi1 - xi0[j]
        assert np.abs(d[:, :2]).max() == 0.0
        assert np.allclose(d[:, 2], -c, rtol=1e-12, atol=1e-12)


def test_drift_limit_below_the_mobility_floor(orc):
    # the mobility is taken at max(|E|, E_floor): the limit must use the same clamp
    cfg = _uniform(1e7, coeffs=dict(D=0.0))
    cfg["coeffs"]["E_floor"] = 2e7
    sim = _seeded(orc, cfg)
    dt, _ = sim.stable_dt({"dt_max": 1.0, "c_drift": 0.3})
    xi0, _, id0 = sim.particles()
    sim.transport(dt)
    xi1, _, id1 = sim.particles()
    o = np.argsort(id0)
    d = xi1 - xi0[o[np.searchsorted(id0, id1, sorter=o)]]
    assert np.allclose(d[:, 2], -0.3, rtol=1e-12, atol=1e-12)


def test_diffusion_limit_spread(orc):
    c_diff = 0.04
    cfg = _uniform(1.0)  # negligible drift: the drift limit does not bind
    sim = _seeded(orc, cfg)
    dt, _ = sim.stable_dt({"dt_max": 1.0, "c_drift": 0.5, "c_diff": c_diff})
    assert dt == pytest.approx(c_diff * cfg["dx"] ** 2 / (2 * cfg["coeffs"]["D"]), rel=1e-14)
    xi0, _, id0 = sim.particles()
    sim.transport(dt)
    xi1, _, id1 = sim.particles()
    o = np.argsort(id0)
    j = o[np.searchsorted(id0, id1, sorter=o)]
    assert np.array_equal(id0[j], id1) and len(id1) > 0.99 * len(id0)
    d = (xi1 - xi0[j]).ravel()
    n = d.size
    # sample variance of 3e4 normal draws: relative sd sqrt(2 / n) < 1%
    assert np.var(d) == pytest.approx(c_diff, rel=5 * np.sqrt(2.0 / n))
    assert abs(d.mean()) < 5 * np.sqrt(c_diff / n) + 1e-9


def test_ionization_limit_mean_fires_per_electron(orc):
    c_ion = 0.02
    cfg = _uniform(1e7, kmc_eps=float("inf"))
    sim = orc.Sim(cfg)
    dt, Em = sim.stable_dt({"dt_max": 1.0, "c_ion": c_ion})
    n, Xe = 2000, 1000
    X = np.zeros((n, 4), dtype=np.int64)
    X[:, 0] = Xe
    k = np.tile(np.asarray(orc.rates(cfg, Em))[:3], (n, 1))
    _, fires = orc.kmc_cells(cfg, X, k, dt, step=0)
    mean = fires[:, 0].sum() / (n * Xe)
    expect_n = n * Xe * c_ion
    assert mean == pytest.approx(c_ion, rel=5 / np.sqrt(expect_n))
    # the binding limit is the ionization one here, not the (off) others
    assert dt < 1.0


def test_limits_off_and_smallest_binds(orc):
    cfg = _uniform(1e7)
    sim = orc.Sim(cfg)
    assert sim.stable_dt({"dt_max": 2e-12})[0] == 2e-12
    a = sim.stable_dt({"dt_max": 1.0, "c_drift": 0.5})[0]
    b = sim.stable_dt({"dt_max": 1.0, "c_diff": 0.5})[0]
    c = sim.stable_dt({"dt_max": 1.0, "c_ion": 0.5})[0]
    both = sim.stable_dt({"dt_max": 1.0, "c_drift": 0.5, "c_diff": 0.5, "c_ion": 0.5})[0]
    assert both == min(a, b, c)
    assert sim.stable_dt({"dt_max": min(a, b, c) / 3, "c_drift": 0.5, "c_diff": 0.5,
                          "c_ion": 0.5})[0] == min(a, b, c) / 3
    # no field: the drift and ionization limits have no rate and are not applied
    z = orc.Sim(_uniform(0.0, coeffs=dict(D=0.0)))
    assert z.stable_dt({"dt_max": 5e-12, "c_drift": 0.5, "c_diff": 0.5, "c_ion": 0.5}) == (5e-12, 0.0)


def _gap(**kw):
    return workloads.preset("streamer_64", grid=(16, 16, 16), dx=1e-3 / 64,
                            seed_centre=(125e-6, 125e-6, 125e-6), seed_sigma=30e-6,
                            V_anode=18e3 * 0.25, **kw)


def test_vacuum_gap_field_bound_is_v_over_l(orc):
    cfg = _gap()
    sim = orc.Sim(cfg)
    L = cfg["grid"][2] * cfg["dx"]
    assert sim.field_max() == pytest.approx(cfg["V_anode"] / L, rel=1e-9)


def test_field_bound_covers_every_particle(orc):
    cfg = _gap()
    sim = orc.Sim(cfg)
    sim.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    sim.step(cfg["dt"], 3)
    Em = sim.field_max()
    _, Ex, Ey, Ez = sim.field()
    xi, _, _ = sim.particles()
    e = np.stack([orc.cic_interp(cfg, g, xi) for g in (Ex, Ey, Ez)], axis=1)
    mag = np.sqrt((e ** 2).sum(axis=1))
    assert mag.max() <= Em * (1 + 1e-12)
    # the space charge makes the field non-uniform: the bound is not just V / L
    assert Em > 1.01 * cfg["V_anode"] / (cfg["grid"][2] * cfg["dx"])


def test_query_does_not_change_the_step(orc):
    cfg = _gap()
    rule = {"dt_max": 1e-12, "c_drift": 0.5, "c_ion": 0.1}
    a = orc.Sim(cfg)
    a.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    dt, _ = a.stable_dt(rule)           # computes the initial field first
    a.step(dt)
    b = orc.Sim(cfg)
    b.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    b.step(dt)                          # the transport computes it itself
    pa, pb = a.particles(), b.particles()
    for u, v in zip(pa, pb):
        assert np.array_equal(u, v)
    # the adaptive driver is the same loop
    c = orc.Sim(cfg)
    c.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    dts = c.step_adaptive(rule, 3)
    d = orc.Sim(cfg)
    d.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    manual = []
    for _ in range(3):
        manual.append(d.stable_dt(rule)[0])
        d.step(manual[-1])
    assert np.array_equal(dts, np.asarray(manual))
    for u, v in zip(c.particles(), d.particles()):
        assert np.array_equal(u, v)
    assert (dts > 0).all() and (dts <= rule["dt_max"]).all()
