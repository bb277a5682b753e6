"""Edge cases through the C ABI, against the FP64 oracle where it applies: empty
inputs, ragged grids (sizes that are not multiples of the 2048-cell scan tiles or the
4096-cell ensemble blocks, odd dimensions), degenerate physics (no field, attachment
only), and capacity limits (reported, state left consistent)."""
import numpy as np
import pytest

from helpers import by_id, gpu_xi, xi_to_cell_off
from paper_2307_01797_amd import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


def _same_as_oracle(g, o, cfg, tol=1e-9, tallies=True):
    cell, off, w, ids = g.particles()
    ids, cell, off, w = by_id(ids, cell, off, w)
    xi_o, w_o, id_o = o.particles()
    id_o, xi_o, w_o = by_id(id_o, xi_o, w_o)
    assert np.array_equal(ids, id_o)
    assert np.array_equal(w.astype(np.uint64), w_o)
    co, _ = xi_to_cell_off(xi_o, cfg["grid"])
    assert np.array_equal(co, cell)
    assert np.abs(gpu_xi(cell, off, cfg["grid"]) - xi_o).max(initial=0.0) < tol
    for k in ("plus", "minus"):
        assert np.array_equal(g.counts(k).astype(np.int64), o.counts(k))
    if not tallies:  # an oracle rebuilt from the GPU state starts its tallies at zero
        return
    dg, do = g.diagnostics(), o.diagnostics()
    for k in ("n_particles", "weight", "n_plus", "n_minus", "outflow_weight", "created",
              "removed_weight", "step"):
        assert dg[k] == do[k], k
    assert dg["fires"] == do["fires"]


def _run_both(itk, orc, cfg, steps):
    g = itk.Sim(cfg, precision="fp64", max_particles=cfg.get("max_particles", 400_000))
    g.seed()
    o = orc.Sim(cfg)
    o.seed_gaussian(cfg["seed_n0"], cfg["seed_centre"], cfg["seed_sigma"])
    g.step(steps)
    o.step(cfg["dt"], steps)
    return g, o


def test_no_particles(itk):
    """A context without particles steps, deposits and reports zeros."""
    for name in ("avalanche_32", "streamer_64"):
        cfg = workloads.preset(name)
        g = itk.Sim(cfg, max_particles=1000)
        g.step(3)
        d = g.diagnostics()
        assert d["n_particles"] == 0 and d["weight"] == 0 and d["step"] == 3
        assert not g.deposit("ngp").any()
        assert g.particles()[0].size == 0
        g.close()


def test_ragged_grid_uniform_field(itk, orc):
    """A 37 x 29 x 23 grid (24679 cells: 12 full scan tiles and a ragged one), seed off
    centre so particles leave through three faces: exact against the oracle."""
    cfg = workloads.preset("avalanche_32", grid=(37, 29, 23), seed_n0=6000,
                           seed_centre=(100e-6, 250e-6, 60e-6), seed_sigma=60e-6)
    g, o = _run_both(itk, orc, cfg, 40)
    _same_as_oracle(g, o, cfg)
    assert g.diagnostics()["outflow_weight"] > 0


def _oracle_from_gpu(orc, cfg, g):
    o = orc.Sim(cfg)
    cell, off, w, ids = g.particles()
    o.set_particles(gpu_xi(cell, off, cfg["grid"]), w.astype(np.uint64), ids)
    for which in ("plus", "minus", "gamma"):
        o.set_counts(which, g.counts(which).astype(np.int64))
    o.set_step(g.diagnostics()["step"])
    return o


def test_ragged_grid_self_consistent(itk, orc):
    """Even but unequal dimensions 40 x 24 x 36 (multigrid coarsens to 10 x 6 x 9), FP64,
    from shared states: the transport (deposit, semi-implicit solve, push) matches the
    oracle's within the solvers' tolerance, and with the same field the react phase
    (photons, sort, KMC, coupling, merge/split) agrees on every integer.  (Free-running
    runs at this size drift apart: both solves stop at a 1e-10 residual, and a field
    difference of that order can flip a merge extent compared in single precision.)"""
    cfg = workloads.preset("streamer_64", grid=(40, 24, 36), dx=1e-3 / 36, V_anode=18e3 * 36 / 64,
                           seed_centre=(20 * 1e-3 / 36, 12 * 1e-3 / 36, 30 * 1e-3 / 36))
    g = itk.Sim(cfg, precision="fp64")
    g.seed()
    g.step(2)
    for _ in range(2):
        o = _oracle_from_gpu(orc, cfg, g)
        o.set_field(g.field())
        g.transport()
        o.transport(cfg["dt"])
        phi_o = o.field()[0]
        assert np.abs(g.field() - phi_o).max() < 1e-8 * np.abs(phi_o).max()
        cell, off, w, ids = g.particles()
        ids, cell, off, w = by_id(ids, cell, off, w)
        xi_o, w_o, id_o = o.particles()
        id_o, xi_o, w_o = by_id(id_o, xi_o, w_o)
        assert np.array_equal(ids, id_o) and np.array_equal(w.astype(np.uint64), w_o)
        assert np.abs(gpu_xi(cell, off, cfg["grid"]) - xi_o).max() < 1e-8
        o = _oracle_from_gpu(orc, cfg, g)
        o.set_efield(g.deposit("ex"), g.deposit("ey"), g.deposit("ez"))
        g.react()
        o.react(cfg["dt"])
        _same_as_oracle(g, o, cfg, tallies=False)
    assert g.diagnostics()["merged_cells"] > 0


def test_zero_field_pure_diffusion(itk, orc):
    """E = 0: no drift and no reactions (alpha, v vanish); only diffusion and removal."""
    cfg = workloads.preset("avalanche_32", E=(0.0, 0.0, 0.0))
    g, o = _run_both(itk, orc, cfg, 30)
    _same_as_oracle(g, o, cfg)
    d = g.diagnostics()
    assert d["fires"] == [0, 0, 0, 0, 0] and d["created"] == 0


def test_attachment_empties_cells(itk, orc):
    """Attachment only (alpha = 0, eta large): cells lose all their electrons, weights
    are removed in ascending id order, and the bank shrinks to nothing."""
    cfg = workloads.preset("avalanche_32", seed_n0=3000,
                           coeffs=dict(alpha_A=0.0, eta=2.0e6))
    g, o = _run_both(itk, orc, cfg, 25)
    _same_as_oracle(g, o, cfg)
    d = g.diagnostics()
    assert d["n_minus"] > 2500 and d["fires"][0] == 0


def test_capacity_reported_and_state_valid(itk):
    """A bank too small for the avalanche's products: the overflow is flagged on the
    device and reported as ECAPACITY by the diagnostics, and the particles that exist
    are valid (cells in range, offsets in [0,1), unique ids)."""
    cfg = workloads.preset("avalanche_32", precision="fp32", E=(0.0, 0.0, 2.0e7))
    g = itk.Sim(cfg, max_particles=12_000)
    g.seed()
    assert g.step_rc(60) == itk.OK
    with pytest.raises(itk.ItokmcError) as err:
        g.diagnostics()
    assert err.value.code == itk.ECAPACITY
    d = g.diagnostics(check=False)
    assert d["overflow"] != 0
    cell, off, w, ids = g.particles()
    assert cell.max() < np.prod(cfg["grid"])
    assert np.all(off >= 0) and np.all(off < 1) and np.all(w > 0)
    assert len(np.unique(ids)) == len(ids)


def test_capacity_with_merging_state_valid(itk):
    """The self-consistent streamer (merging on) in a bank only a little larger than its
    seed: KMC products that find no slot are flagged, the coupling still merges the
    cells whose products it makes itself, and every particle left is valid (cells in
    range, offsets in [0,1), positive weights, unique ids)."""
    from test_gpu_parity import _streamer_small
    cfg = _streamer_small(precision="fp32", gmg_rtol=1e-10)
    probe = itk.Sim(cfg, precision="fp32")
    probe.seed()
    n0 = probe.diagnostics()["n_particles"]
    del probe
    g = itk.Sim(cfg, precision="fp32", max_particles=n0 + 400)
    g.seed()
    assert g.step_rc(12) == itk.OK
    with pytest.raises(itk.ItokmcError) as err:
        g.diagnostics()
    assert err.value.code == itk.ECAPACITY
    d = g.diagnostics(check=False)
    assert d["overflow"] & 1 and d["merged_cells"] > 0
    cell, off, w, ids = g.particles()
    assert len(cell) > 0 and cell.max() < np.prod(cfg["grid"])
    assert np.all(off >= 0) and np.all(off < 1) and np.all(w > 0)
    assert len(np.unique(ids)) == len(ids)


def test_ensemble_empty_and_ragged(itk):
    """An ensemble step with no realizations; a realization with no electrons; a ragged
    grid (33 x 17 x 9 = 5049 cells: one full 4096-cell block and a partial one) alone
    and as a plain context."""
    ens = itk.Ensemble(4, 1 << 16, 200_000)
    ens.step(2)
    assert ens.poll() == []
    base = workloads.ensemble_realization(3)
    empty = dict(base, grid=(32, 32, 32), seed_n0=0, steps=5, max_particles=10_000)
    L = np.array([33, 17, 9]) * base["dx"]
    ragged = dict(base, grid=(33, 17, 9), seed_n0=2000, seed_centre=tuple(L / 2),
                  seed_sigma=0.2 * float(L.min()), steps=30, stop_particles=0,
                  max_particles=100_000)
    s0 = ens.admit(empty)
    s1 = ens.admit(ragged)
    done = {}
    for _ in range(100):
        ens.step(1)
        for slot, state, tag, steps in ens.poll():
            done[slot] = steps
        if len(done) == 2:
            break
    assert done[s0] == 5 and ens.result(s0)["n_particles"] == 0
    g = itk.Sim(ragged, max_particles=ragged["max_particles"])
    g.seed()
    g.step(30)
    c1, o1, w1, i1 = ens.particles(s1)
    c2, o2, w2, i2 = g.particles()
    i1, c1, o1, w1 = by_id(i1, c1, o1, w1)
    i2, c2, o2, w2 = by_id(i2, c2, o2, w2)
    assert np.array_equal(i1, i2) and np.array_equal(c1, c2) and np.array_equal(w1, w2)
    assert np.array_equal(o1, o2)


def test_rho_selector_matches_oracle(itk, orc):
    """ITOKMC_Q_RHO: e (n+ - n-)/dV - e n_e(CIC) of the current state, against the
    oracle's charge density of the same particles and ion counts."""
    cfg = workloads.preset("streamer_64", grid=(20, 18, 24), dx=1e-3 / 64)
    rng = np.random.default_rng(12)
    n = 5000
    xi = rng.random((n, 3)) * np.array(cfg["grid"])
    w = rng.integers(1, 3000, size=n).astype(np.uint64)
    ids = np.arange(n, dtype=np.uint64) * np.uint64(3) + np.uint64(11)
    ncell = int(np.prod(cfg["grid"]))
    npl = rng.integers(0, 4000, ncell)
    nmi = rng.integers(0, 300, ncell)
    cell, off = xi_to_cell_off(xi, cfg["grid"])
    o = orc.Sim(cfg)
    o.set_particles(xi, w, ids)
    o.set_counts("plus", npl)
    o.set_counts("minus", nmi)
    want = o.charge_density()
    for prec, tol in (("fp64", 1e-12), ("fp32", 1e-6)):
        g = itk.Sim(cfg, precision=prec, max_particles=2 * n)
        g.set_particles(cell, off, w.astype(np.uint32), ids)
        g.set_counts("plus", npl.astype(np.uint32))
        g.set_counts("minus", nmi.astype(np.uint32))
        got = g.deposit("rho")
        scale = np.abs(want).max()
        assert np.abs(got - want).max() <= tol * scale, (prec, np.abs(got - want).max() / scale)
        g.close()


def test_solver_nonconvergence_reported(itk):
    """A field solve limited to one multigrid cycle misses the 1e-10 tolerance: the
    step returns ENOCONV and the state stays usable (the best potential is kept)."""
    cfg = workloads.preset("streamer_64", grid=(32, 32, 32), dx=1e-3 / 32, gmg_max_cycles=1)
    g = itk.Sim(cfg, max_particles=500_000)
    g.seed()
    rc = g.step_rc(1)
    assert rc == itk.ENOCONV, rc
    d = g.diagnostics(check=False)
    assert d["solver_cycles"] == 1 and d["solver_relres"] > 1e-10
    phi = g.field()
    assert np.all(np.isfinite(phi))
    g.close()


def test_nan_coefficients_rejected(itk):
    """set_coefficients keeps the previous set and returns EINVAL for a NaN."""
    import ctypes
    import math
    cfg = workloads.preset("avalanche_32", seed_n0=500)
    g = itk.Sim(cfg, max_particles=10_000)
    c = itk.make_coeffs(cfg)
    c.D = math.nan
    assert itk.lib().itokmc_set_coefficients(g.h, ctypes.byref(c)) == itk.EINVAL
    g.seed()
    g.step(2)                      # the earlier coefficients are still in force
    assert g.diagnostics()["step"] == 2
    g.close()


def test_oversized_cell_reported_as_capacity(itk):
    """A cell holding more particles than the largest merge staging is left unmerged
    and flagged (ITOKMC_OVF_MERGE): diagnostics returns ECAPACITY and counts the cell;
    the other cells are merged as usual."""
    cfg = workloads.preset("avalanche_32", grid=(8, 8, 8), n_ppc=32, E=(0.0, 0.0, 1.0),
                           coeffs=dict(alpha_A=0.0, eta=0.0, D=0.0), precision="fp32")
    rng = np.random.default_rng(3)
    big, small = 2000, 100
    cell = np.concatenate([np.full(big, 100), np.full(small, 300)]).astype(np.uint32)
    off = rng.random((big + small, 3)) * 0.98 + 0.01
    w = np.ones(big + small, dtype=np.uint32)
    ids = np.arange(big + small, dtype=np.uint64) + np.uint64(1)
    g = itk.Sim(cfg, max_particles=20_000)
    g.set_particles(cell, off, w, ids)
    g.step(1)
    with pytest.raises(itk.ItokmcError) as err:
        g.diagnostics()
    assert err.value.code == itk.ECAPACITY
    d = g.diagnostics(check=False)
    assert d["overflow"] & itk.OVF_MERGE and d["merge_skipped"] == 1
    c2, _, w2, _ = g.particles()
    assert np.sum(c2 == 100) == big and np.sum(c2 == 300) == 32
    assert int(w2.sum()) == big + small
    g.close()
