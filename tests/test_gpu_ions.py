"""The library's mobile ions (the lattice jump process of the header's ion-transport
paragraph) against the oracle's: ion counts and their outflow tallies bit-exact, with
the electrons, fires and positions under the usual bars: ion clouds in a prescribed
field (FP64 and FP32: the hop rates come from the same field on both sides), the FP64
avalanche free-running, a charged ion sheet in its own solved field, and the FP64
self-consistent streamer free-running (each side's own E^{k+1})."""
import numpy as np
import pytest

from paper_2307_01797_amd import workloads
from test_gpu_parity import _compare, _compare_tallies, _streamer_small

pytestmark = pytest.mark.gpu

# exaggerated ion transport, so that ions cross many faces within a short run
FAST_IONS = dict(mu_ion=3e-2, D_ion=5e-3)


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


def _tallies(g, o):
    dg, do = g.diagnostics(), o.diagnostics()
    for key in ("ion_outflow_plus", "ion_outflow_minus"):
        assert dg[key] == do[key], (key, dg[key], do[key])
    return dg


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_ion_cloud_in_prescribed_field(itk, orc, prec):
    """Ions only (no electrons), random counts, a tilted uniform field, large hop
    probabilities: the same rates on both sides, so every count and tally is exact."""
    cfg = workloads.preset("avalanche_32", grid=(12, 10, 14), E=(2e6, -1e6, 1.5e7), precision=prec,
                           coeffs=FAST_IONS)
    rng = np.random.default_rng(11)
    n = 12 * 10 * 14
    p = rng.integers(0, 3000, n) * (rng.random(n) < 0.6)
    m = rng.integers(0, 300, n) * (rng.random(n) < 0.6)
    g = itk.Sim(cfg, precision=prec, max_particles=1000)
    g.set_particles(np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint64))
    g.set_counts("plus", p.astype(np.uint32))
    g.set_counts("minus", m.astype(np.uint32))
    o = orc.Sim(cfg)
    o.set_counts("plus", p)
    o.set_counts("minus", m)
    for dt in (1e-12, 2e-11, 2e-10, 2e-10):
        g.transport(dt)
        o.transport(dt)
        for which in ("plus", "minus"):
            assert np.array_equal(g.counts(which).astype(np.int64), o.counts(which)), (which, dt)
        _tallies(g, o)
    d = g.diagnostics()
    assert d["ion_outflow_plus"] > 0 and d["ion_outflow_minus"] > 0
    assert g.counts("plus").sum() + d["ion_outflow_plus"] == p.sum()


def test_avalanche_with_mobile_ions_fp64(itk, orc):
    cfg = workloads.preset("avalanche_32", E=(0.0, 0.0, 1.5e7), coeffs=FAST_IONS)
    g = itk.Sim(cfg, precision="fp64")
    g.seed()
    q0 = g.diagnostics()["charge"]
    o = orc.Sim(cfg)
    o.seed_gaussian(cfg["seed_n0"], cfg["seed_centre"], cfg["seed_sigma"])
    for target in (1, 10, 40):
        n = target - g.diagnostics()["step"]
        g.step(n)
        o.step(cfg["dt"], n)
        for which in ("plus", "minus"):
            assert np.array_equal(g.counts(which).astype(np.int64), o.counts(which)), which
        d = _tallies(g, o)
        assert _compare(g, o, cfg, 1e-9) == 0
        _compare_tallies(g, o)
    assert d["ion_outflow_plus"] > 0
    assert d["charge"] == q0 + d["outflow_weight"] - d["ion_outflow_plus"] + d["ion_outflow_minus"]


def test_ion_sheet_self_consistent(itk, orc):
    """A sheet of positive ions in a plane gap, no electrons, FP64: one transport solves
    for the sheet's field and moves the ions with it; counts equal the oracle's."""
    nx, ny, nz, L, V = 4, 4, 32, 1e-3, 2e3
    cfg = workloads.preset("streamer_64", grid=(nx, ny, nz), dx=L / nz, V_anode=V, n_ppc=0,
                           gmg_rtol=1e-12, coeffs=dict(mu_ion=2e-4, D_ion=0.0))
    p = np.zeros(nx * ny * nz, dtype=np.int64)
    p[12 * nx * ny:13 * nx * ny] = 2_000_000
    g = itk.Sim(cfg, precision="fp64", max_particles=1000)
    g.set_particles(np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint64))
    g.set_counts("plus", p.astype(np.uint32))
    o = orc.Sim(cfg)
    o.set_counts("plus", p)
    g.transport(2e-9)
    o.transport(2e-9)
    assert np.array_equal(g.counts("plus").astype(np.int64), o.counts("plus"))
    moved = (g.counts("plus").astype(np.int64) != p).sum()
    assert moved >= 2 * nx * ny


def test_streamer_with_mobile_ions_fp64(itk, orc):
    cfg = _streamer_small(coeffs=FAST_IONS)
    g = itk.Sim(cfg, precision="fp64")
    g.seed()
    o = orc.Sim(cfg)
    o.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    for target in (1, 3, 6):
        n = target - g.diagnostics()["step"]
        g.step(n)
        o.step(cfg["dt"], n)
        assert _compare(g, o, cfg, 1e-9) == 0
        _compare_tallies(g, o)
        _tallies(g, o)
    # the ions moved: the counts differ from a run with immobile ions
    h = itk.Sim(_streamer_small(), precision="fp64")
    h.seed()
    h.step(6)
    assert not np.array_equal(h.counts("plus"), g.counts("plus"))


def test_stop_rule_with_mobile_ions(itk):
    """The device-side stop rule halts the ion passes with the rest of the step: the
    state after step_until equals the host-checked run of the same number of steps."""
    cfg = workloads.preset("avalanche_32", E=(0.0, 0.0, 1.5e7), precision="fp32", coeffs=FAST_IONS)
    a = itk.Sim(cfg, precision="fp32")
    a.seed()
    done = a.step_until(40, stop_particles=12_000)
    assert 0 < done < 40
    b = itk.Sim(cfg, precision="fp32")
    b.seed()
    b.step(done)
    for which in ("plus", "minus"):
        assert np.array_equal(a.counts(which), b.counts(which))
    assert a.diagnostics()["ion_outflow_plus"] == b.diagnostics()["ion_outflow_plus"]


def test_ensemble_rejects_mobile_ions(itk):
    cfg = workloads.ensemble_realization(0)
    cfg["coeffs"].update(FAST_IONS)
    ens = itk.Ensemble(2, 1 << 20, 1_000_000)
    with pytest.raises(itk.ItokmcError) as e:
        ens.admit(cfg)
    assert e.value.code == itk.EINVAL and "mobile ions" in str(e.value)


def test_ragged_grid_ion_cloud(itk, orc):
    """Mobile ions on a 37 x 29 x 23 grid (no dimension a multiple of any tile), ions on
    every face of the box, FP32: counts and tallies exact."""
    cfg = workloads.preset("avalanche_32", grid=(37, 29, 23), E=(-3e6, 4e6, 1.2e7), precision="fp32",
                           coeffs=FAST_IONS)
    rng = np.random.default_rng(17)
    n = 37 * 29 * 23
    p = rng.integers(0, 400, n)
    m = rng.integers(0, 40, n)
    g = itk.Sim(cfg, precision="fp32", max_particles=1000)
    g.set_particles(np.zeros(0), np.zeros((0, 3)), np.zeros(0), np.zeros(0, np.uint64))
    g.set_counts("plus", p.astype(np.uint32))
    g.set_counts("minus", m.astype(np.uint32))
    o = orc.Sim(cfg)
    o.set_counts("plus", p)
    o.set_counts("minus", m)
    for _ in range(3):
        g.step(1, dt=5e-11)
        o.step(5e-11)
        for which in ("plus", "minus"):
            assert np.array_equal(g.counts(which).astype(np.int64), o.counts(which)), which
        _tallies(g, o)


def test_next_step_features_together_fp64(itk, orc):
    """The 16^3 self-consistent streamer with the TSC shape, recombination, mobile ions
    and the dynamic time step at once, FP64, free-running: every integer exact, the step
    sizes within 1e-9, positions within 1e-9 cells."""
    from test_gpu_parity import _recomb
    coeffs = dict(_recomb(1e7), **FAST_IONS)
    cfg = _streamer_small(shape="tsc", coeffs=coeffs)
    rule = {"dt_max": 1e-12, "c_drift": 0.2, "c_ion": 0.05}
    g = itk.Sim(cfg, precision="fp64")
    g.seed()
    o = orc.Sim(cfg)
    o.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    for n in (1, 2, 2):
        dg = g.step_adaptive(rule, n)
        do = o.step_adaptive(rule, n)
        assert np.allclose(dg, do, rtol=1e-9, atol=0)
        assert _compare(g, o, cfg, 1e-9) == 0
        _compare_tallies(g, o)
        _tallies(g, o)
    d = g.diagnostics()
    assert d["fires"][3] > 0 and d["step"] == 5
