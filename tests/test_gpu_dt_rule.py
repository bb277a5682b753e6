"""The library's dynamic time-step rule (itokmc_stable_dt, itokmc_step_adaptive) against
the oracle's: the field bound and dt of each query, and free-running adaptive runs whose
every step takes its own dt (the rule's reading is in the oracle's sim.c and the
header).  Bars as in the other parity tests: integers bit-exact, FP64 positions within
1e-9 cells, dt and the field bound within the solver's agreement (1e-9) in the
self-consistent mode and equal in the prescribed-field mode (host arithmetic on both
sides)."""
import numpy as np
import pytest

from helpers import by_id, gpu_xi
from paper_2307_01797_amd import workloads
from test_gpu_parity import _compare, _compare_tallies, _oracle_from_gpu, _streamer_small

pytestmark = pytest.mark.gpu

RULES = [
    {"dt_max": 1.0, "c_drift": 0.5},
    {"dt_max": 1.0, "c_diff": 0.04},
    {"dt_max": 1.0, "c_ion": 0.02},
    {"dt_max": 3e-13, "c_drift": 0.5, "c_diff": 0.5, "c_ion": 0.5},
    {"dt_max": 1.0, "c_drift": 0.3, "c_diff": 0.2, "c_ion": 0.05},
]


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_prescribed_field_rule_equals_oracle(itk, orc, prec):
    for E in (1e5, 3e6, 1e7, 3e7):
        cfg = workloads.preset("avalanche_32", E=(0.0, 0.3 * E, 0.954 * E), precision=prec)
        g = itk.Sim(cfg, precision=prec, max_particles=1000)
        o = orc.Sim(cfg)
        for r in RULES:
            dg, eg = g.stable_dt(r)
            do, eo = o.stable_dt(r)
            assert eg == pytest.approx(eo, rel=1e-15) and dg == pytest.approx(do, rel=1e-14), (E, r)


def test_avalanche_fp64_adaptive_free_running(itk, orc):
    cfg = workloads.preset("avalanche_32")
    rule = {"dt_max": 2e-12, "c_drift": 0.3, "c_ion": 0.01}
    g = itk.Sim(cfg, precision="fp64")
    g.seed()
    o = orc.Sim(cfg)
    o.seed_gaussian(cfg["seed_n0"], cfg["seed_centre"], cfg["seed_sigma"])
    for n in (1, 4, 10):
        dg = g.step_adaptive(rule, n)
        do = o.step_adaptive(rule, n)
        assert np.allclose(dg, do, rtol=1e-14, atol=0)
        assert _compare(g, o, cfg, 1e-9) == 0
        _compare_tallies(g, o)
    # the binding limit is not dt_max: the rule chose the step
    assert dg.max() < rule["dt_max"]


def test_streamer_fp64_adaptive_free_running(itk, orc):
    """Self-consistent 16^3 streamer seed, FP64: the first query computes the initial
    field on both sides; each step's dt comes from that side's own E^k."""
    cfg = _streamer_small()
    rule = {"dt_max": 2e-12, "c_drift": 0.2, "c_ion": 0.05}
    g = itk.Sim(cfg, precision="fp64")
    g.seed()
    o = orc.Sim(cfg)
    o.seed_neutral(cfg["seed_peak"], cfg["seed_centre"], cfg["seed_sigma"])
    dg, eg = g.stable_dt(rule)
    do, eo = o.stable_dt(rule)
    assert eg == pytest.approx(eo, rel=1e-9) and dg == pytest.approx(do, rel=1e-9)
    for n in (1, 2, 3):
        dts_g = g.step_adaptive(rule, n)
        dts_o = o.step_adaptive(rule, n)
        assert np.allclose(dts_g, dts_o, rtol=1e-9, atol=0)
        assert _compare(g, o, cfg, 1e-9) == 0
        _compare_tallies(g, o)
    assert g.diagnostics()["step"] == 6


def test_streamer_fp32_field_bound_from_the_same_field(itk, orc):
    """FP32 context after a few steps: the oracle given the GPU's stored field finds the
    same bound (both take the squares in double from the same single-precision values)."""
    cfg = _streamer_small(precision="fp32", gmg_rtol=1e-10)
    g = itk.Sim(cfg, precision="fp32")
    g.seed()
    g.step(3)
    o = _oracle_from_gpu(orc, cfg, g)
    o.set_efield(g.deposit("ex"), g.deposit("ey"), g.deposit("ez"))
    rule = {"dt_max": 1.0, "c_drift": 0.25}
    dg, eg = g.stable_dt(rule)
    do, eo = o.stable_dt(rule)
    assert eg == pytest.approx(eo, rel=1e-15) and dg == pytest.approx(do, rel=1e-14)
    # and it bounds every particle's interpolated field
    cell, off, _, _ = g.particles()
    xi = gpu_xi(cell, off, cfg["grid"])
    e = np.stack([orc.cic_interp(cfg, g.deposit(a), xi) for a in ("ex", "ey", "ez")], axis=1)
    assert np.sqrt((e ** 2).sum(axis=1)).max() <= eg * (1 + 1e-12)


def test_query_before_the_first_step_changes_nothing(itk):
    """The query's initial solve replaces the first transport's: the step that follows
    is bit-identical to the same step without the query."""
    cfg = _streamer_small(precision="fp32", gmg_rtol=1e-10)
    rule = {"dt_max": 1e-12, "c_drift": 0.2}
    a = itk.Sim(cfg, precision="fp32")
    a.seed()
    dt, _ = a.stable_dt(rule)
    a.step(1, dt=dt)
    b = itk.Sim(cfg, precision="fp32")
    b.seed()
    b.step(1, dt=dt)
    # the bank order inside a cell is not fixed (atomic ranks): compare by id
    pa, pb = a.particles(), b.particles()
    for u, v in zip(by_id(pa[3], *pa[:3]), by_id(pb[3], *pb[:3])):
        assert np.array_equal(u, v)
    assert np.array_equal(a.field(), b.field())


def test_rule_validation(itk):
    cfg = workloads.preset("avalanche_32")
    g = itk.Sim(cfg, precision="fp32", max_particles=1000)
    for bad in ({"dt_max": 0.0}, {"dt_max": -1e-12}, {"dt_max": float("nan")},
                {"dt_max": 1e-12, "c_drift": -0.1}, {"dt_max": 1e-12, "c_ion": float("inf")}):
        with pytest.raises(itk.ItokmcError):
            g.stable_dt(bad)
    steep = workloads.preset("avalanche_32", coeffs=dict(mu_b=-1.5))
    h = itk.Sim(steep, precision="fp32", max_particles=1000)
    with pytest.raises(itk.ItokmcError):
        h.stable_dt({"dt_max": 1e-12, "c_drift": 0.5})
    assert h.stable_dt({"dt_max": 1e-12, "c_diff": 0.5})[0] > 0.0
