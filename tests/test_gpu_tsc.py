"""The library's quadratic B-spline (TSC) shape (conductivity and charge deposits, field
interpolation, ions spread like the electrons) against the oracle's and against the
one-dimensional closed form of tsc_layer_case.py.  Bars as in the other parity tests:
integers bit-exact, FP64 positions within 1e-9 cells, FP32 positions within 1e-5 cells
outside the tie band."""
import numpy as np
import pytest

from helpers import by_id
from paper_2307_01797_amd import workloads
from semi_implicit_case import ez_column
from test_gpu_parity import _compare, _compare_tallies, _oracle_from_gpu, _streamer_small
from tsc_layer_case import make_layer

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def itk():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    from paper_2307_01797_amd import itokmc
    itokmc.lib()
    return itokmc


@pytest.mark.parametrize("prec,ftol,ptol", [("fp64", 1e-8, 1e-10), ("fp32", 2e-6, 2e-7)])
def test_layer_closed_form_gpu(itk, prec, ftol, ptol):
    c = make_layer(workloads.preset("streamer_64"), "tsc")
    cfg, grid = c["cfg"], c["cfg"]["grid"]
    print(f"tsc layer {prec} grid={grid}", flush=True)
    g = itk.Sim(cfg, precision=prec, max_particles=len(c["ids"]) * 4)
    g.set_particles(c["cell"], c["xi"] - np.floor(c["xi"]), c["w"].astype(np.uint32), c["ids"])
    g.set_counts("plus", c["nplus"].astype(np.uint32))
    # the neutral layer has no charge with the ions spread like the electrons
    assert np.abs(g.deposit("rho")).max() <= 1e-12 * 1.602e-19 * c["w"][0] / c["dx"] ** 3
    g.transport(cfg["dt"])
    Eh = np.abs(c["Ez_col"]).max()
    col, spread = ez_column(g.deposit("ez"), grid)
    assert np.abs(col - c["Ez_col"]).max() <= ftol * Eh
    assert spread.max() <= ftol * Eh
    assert np.abs(g.deposit("ex")).max() <= ftol * Eh and np.abs(g.deposit("ey")).max() <= ftol * Eh
    cell, off, w, ids = g.particles()
    o, p = np.argsort(ids), np.argsort(c["ids"])
    assert np.array_equal(ids[o], c["ids"][p])
    nx, ny, _ = grid
    ijk = np.stack([cell % nx, (cell // nx) % ny, cell // (nx * ny)], 1).astype(np.float64)
    d = (ijk + off)[o] - c["xi"][p]
    assert np.abs(d[:, :2]).max() <= ptol
    assert np.abs(d[:, 2] - c["dz"][p]).max() <= ptol


def test_streamer_tsc_fp64_free_running(itk, orc):
    """Self-consistent 16^3 streamer seed with the TSC shape, free-running FP64: every
    integer agrees, positions to 1e-9 cells; the shape changes the result (against the
    same run with CIC)."""
    cfg = _streamer_small(shape="tsc")
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
    assert g.diagnostics()["merged_cells"] > 0
    phi_o = o.field()[0]
    assert np.abs(g.field() - phi_o).max() < 1e-9 * np.abs(phi_o).max()
    h = itk.Sim(_streamer_small(), precision="fp64")
    h.seed()
    h.step(6)
    assert np.abs(h.field() - g.field()).max() > 1e-6 * np.abs(phi_o).max()


def test_streamer_tsc_fp32_resync(itk, orc):
    """FP32 with the TSC shape, each transport from an identical state: potential within
    1e-6 of its range, positions within 1e-5 cells outside the tie band; react exact."""
    cfg = _streamer_small(precision="fp32", gmg_rtol=1e-10, shape="tsc")
    g = itk.Sim(cfg, precision="fp32")
    g.seed()
    g.step(3)
    nband = 0
    for _ in range(3):
        o = _oracle_from_gpu(orc, cfg, g)
        o.set_field(g.field())
        o.set_efield(g.deposit("ex"), g.deposit("ey"), g.deposit("ez"))
        g.transport()
        o.transport(cfg["dt"])
        phi_g, phi_o = g.field(), o.field()[0]
        assert np.abs(phi_g - phi_o).max() < 1e-6 * np.abs(phi_o).max()
        nband += _compare(g, o, cfg, 1e-5, band=1e-5)
        o = _oracle_from_gpu(orc, cfg, g)
        o.set_efield(g.deposit("ex"), g.deposit("ey"), g.deposit("ez"))
        g.react()
        o.react(cfg["dt"])
        assert _compare(g, o, cfg, 2e-6) == 0
    assert nband <= 2


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_density_and_charge_queries(itk, orc, prec):
    cfg = _streamer_small(shape="tsc", precision=prec)
    g = itk.Sim(cfg, precision=prec)
    g.seed()
    g.step(2)
    o = _oracle_from_gpu(orc, cfg, g)
    n_o, rho_o = o.cic_density(), o.charge_density()
    n_g, rho_g = g.deposit("cic"), g.deposit("rho")
    assert np.abs(n_g - n_o).max() <= 1e-12 * np.abs(n_o).max()
    scale = 1.602176634e-19 * np.abs(n_o).max()
    assert np.abs(rho_g - rho_o).max() <= 1e-12 * scale
    # the density spreads over more cells than CIC would give
    cic = dict(cfg, shape="cic")
    assert np.count_nonzero(n_o) > np.count_nonzero(_oracle_from_gpu(orc, cic, g).cic_density())


def test_tsc_run_is_reproducible(itk):
    cfg = _streamer_small(precision="fp32", gmg_rtol=1e-10, shape="tsc")
    out = []
    for _ in range(2):
        g = itk.Sim(cfg, precision="fp32")
        g.seed()
        g.step(4)
        cell, off, w, ids = g.particles()
        out.append(by_id(ids, cell, off, w) + (g.field(),))
    for a, b in zip(*out):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 1e-6)])
def test_ragged_walls_many_per_cell(itk, orc, prec, tol):
    """TSC on a 13 x 11 x 9 grid with clusters of particles in cells on every wall and
    corner (runs of equal cells in the wavefronts, clamped and folded nodes) and random
    ion counts: one transport, the potential against the oracle's from the same state,
    and the charge-density query exact to rounding."""
    grid = (13, 11, 9)
    cfg = _streamer_small(grid=grid, shape="tsc", precision=prec, n_ppc=0, gmg_rtol=1e-12)
    rng = np.random.default_rng(29)
    nx, ny, nz = grid
    cells = []
    for i in (0, nx // 2, nx - 1):
        for j in (0, ny // 2, ny - 1):
            for k in (0, nz // 2, nz - 1):
                cells += [i + nx * (j + ny * k)] * int(rng.integers(1, 9))
    cells = np.sort(np.array(cells, dtype=np.int64))
    n = len(cells)
    off = rng.random((n, 3))
    w = rng.integers(1, 2000, n).astype(np.uint32)
    ids = np.arange(1, n + 1, dtype=np.uint64) * 7919
    g = itk.Sim(cfg, precision=prec, max_particles=4 * n)
    g.set_particles(cells, off, w, ids)
    nc = nx * ny * nz
    p = rng.integers(0, 3000, nc) * (rng.random(nc) < 0.3)
    m = rng.integers(0, 300, nc) * (rng.random(nc) < 0.3)
    g.set_counts("plus", p.astype(np.uint32))
    g.set_counts("minus", m.astype(np.uint32))
    o = _oracle_from_gpu(orc, cfg, g)
    rho_o = o.charge_density()
    scale = 1.602176634e-19 * np.abs(o.cic_density()).max()
    assert np.abs(g.deposit("rho") - rho_o).max() <= 1e-12 * max(scale, np.abs(rho_o).max())
    g.transport(cfg["dt"])
    o.transport(cfg["dt"])
    phi_g, phi_o = g.field(), o.field()[0]
    assert np.abs(phi_g - phi_o).max() <= tol * np.abs(phi_o).max()
