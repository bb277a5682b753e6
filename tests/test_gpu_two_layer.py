"""The GPU's semi-implicit step (section "Semi-implicit Euler-Maruyama method", eqs.
poisson_simp and conductivity) against the two-layer closed form: a neutral plasma on
the cell centres of the lower half of the gap, D = 0.  The step's field must be the
layered dielectric solution with eps_l = 1 + e mu(V/L) n dt / eps0, and every electron
must move by -mu(V/L) E^{k+1} dt (see semi_implicit_case.py).  Bars: the field within
1e-8 of E_h in double precision (the multigrid stops at a relative residual of 1e-10)
and 2e-6 in single; displacements within 1e-10 and 2e-7 cells."""
import numpy as np
import pytest

from paper_2307_01797_amd import workloads

from semi_implicit_case import ez_column, make_case

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec,ftol,ptol", [("fp64", 1e-8, 1e-10), ("fp32", 2e-6, 2e-7)])
@pytest.mark.parametrize("eps_jump", [0.5, 3.0])
def test_two_layer_closed_form_gpu(prec, ftol, ptol, eps_jump):
    import torch
    assert torch.cuda.is_available()
    from paper_2307_01797_amd import itokmc
    c = make_case(workloads.preset("streamer_64"), eps_jump=eps_jump)
    cfg, grid = c["cfg"], c["cfg"]["grid"]
    print(f"two-layer {prec} eps_jump={eps_jump} grid={grid}", flush=True)
    g = itokmc.Sim(cfg, precision=prec, max_particles=len(c["ids"]) * 4)
    off = c["xi"] - np.floor(c["xi"])
    g.set_particles(c["cell"], off, c["w"].astype(np.uint32), c["ids"])
    g.set_counts("plus", c["nplus"].astype(np.uint32))
    g.transport(cfg["dt"])
    E_h = c["E_h"]
    Ex, Ey, Ez = g.deposit("ex"), g.deposit("ey"), g.deposit("ez")
    col, spread = ez_column(Ez, grid)
    assert np.abs(col - c["Ez_col"]).max() <= ftol * E_h, np.abs(col - c["Ez_col"]).max() / E_h
    assert spread.max() <= ftol * E_h
    assert np.abs(Ex).max() <= ftol * E_h and np.abs(Ey).max() <= ftol * E_h
    cell, off2, w, ids = g.particles()
    assert len(ids) == len(c["ids"])
    o, p = np.argsort(ids), np.argsort(c["ids"])
    assert np.array_equal(ids[o], c["ids"][p])
    assert np.array_equal(w[o].astype(np.uint64), c["w"][p])
    nx, ny, _ = grid
    ijk = np.stack([cell % nx, (cell // nx) % ny, cell // (nx * ny)], 1).astype(np.float64)
    d = (ijk + off2)[o] - c["xi"][p]
    assert np.abs(d[:, :2]).max() <= ptol
    assert np.abs(d[:, 2] - c["dz"][p]).max() <= ptol, np.abs(d[:, 2] - c["dz"][p]).max()
