"""A closed-form case of the semi-implicit field coupling (section "Semi-implicit
Euler-Maruyama method", eqs. poisson_simp and conductivity, final algorithm steps 1-5),
shared by the oracle pin and the GPU test.  Index bookkeeping and the analytic solution
only; none of the method's code.

Set-up: a plane gap (phi = 0 at z = 0, phi = V at z = L, Neumann on x and y) whose lower
half holds a neutral plasma: one electron of weight w at the centre of every cell with
k < nz/2 and w positive ions in the same cell, D = 0 (so X_dagger = X^k).  The charge is
zero, so the initial field is the vacuum field V/L and every electron has mobility
mu(V/L).  Step 1 deposits sigma = e mu(V/L) w / dV in the lower half, so the step's
solve sees two dielectric layers eps_l = 1 + sigma dt / eps0 (below) and eps_h = 1.  The
flux eps E is the same through every z face, and the two layers split the voltage:
    eps_l E_l = E_h,   (E_l + E_h) L / 2 = V.
The cell-centred potential is then exactly linear in each layer, and E by central
differences is E_l in the lower layer, E_h in the upper one, and (3 E_l + E_h)/4,
(E_l + 3 E_h)/4 in the two cells next to the interface.  Steps 4-5 move each electron
(which sits on a cell centre, where interpolation returns the cell's own value) by
-mu(V/L) E^{k+1} dt along z."""
import numpy as np

E_CHARGE = 1.602176634e-19
EPS0 = 8.8541878128e-12


def make_case(cfg_base, grid=(8, 8, 32), L=1e-3, V=18e3, eps_jump=1.0, dt=0.5e-12):
    nx, ny, nz = grid
    dx = L / nz
    cfg = dict(cfg_base)
    cfg.update(name="two_layer", grid=grid, dx=dx, V_anode=V, field="poisson", dt=dt,
               n_ppc=0, coeffs=dict(cfg_base["coeffs"], D=0.0, kgamma_ratio=0.0))
    mu_a, mu_E0, mu_b = (cfg["coeffs"][k] for k in ("mu_a", "mu_E0", "mu_b"))
    mu = mu_a * (max(V / L, cfg["coeffs"]["E_floor"]) / mu_E0) ** mu_b
    dV = dx ** 3
    # weight per cell that makes sigma dt / eps0 = eps_jump
    w = int(round(eps_jump * EPS0 * dV / (E_CHARGE * mu * dt)))
    k_lo = np.arange(nz // 2)
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), k_lo, indexing="ij")
    ijk = np.stack([ii.ravel(), jj.ravel(), kk.ravel()], axis=1)
    xi = ijk + 0.5
    cell = (ijk[:, 0] + nx * (ijk[:, 1] + ny * ijk[:, 2])).astype(np.uint32)
    n = len(cell)
    ids = np.arange(1, n + 1, dtype=np.uint64) * np.uint64(977)
    weights = np.full(n, w, dtype=np.uint64)
    nplus = np.zeros(nx * ny * nz, dtype=np.int64)
    nplus[cell] = w
    # closed form
    sigma = E_CHARGE * mu * w / dV
    eps_l = 1.0 + sigma * dt / EPS0
    E_l = 2.0 * V / (L * (1.0 + eps_l))
    E_h = eps_l * E_l
    Ez = np.empty(nz)
    Ez[: nz // 2] = -E_l
    Ez[nz // 2:] = -E_h
    Ez[nz // 2 - 1] = -(3 * E_l + E_h) / 4
    Ez[nz // 2] = -(E_l + 3 * E_h) / 4
    dz = -mu * Ez[ijk[:, 2]] * dt / dx   # grid units
    return dict(cfg=cfg, xi=xi, cell=cell, ids=ids, w=weights, nplus=nplus, mu=mu,
                eps_l=eps_l, E_l=E_l, E_h=E_h, Ez_col=Ez, dz=dz, dx=dx, ijk=ijk)


def ez_column(Ez_cells, grid):
    """Per-z mean and spread of a cell-centred field over each x-y plane."""
    nx, ny, nz = grid
    a = np.asarray(Ez_cells).reshape(nz, ny, nx)
    return a.mean(axis=(1, 2)), (a.max(axis=(1, 2)) - a.min(axis=(1, 2)))

