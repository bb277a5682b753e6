"""A closed form of the semi-implicit step with the quadratic B-spline (TSC) shape,
shared by the oracle pin and the GPU test.  Index bookkeeping and the analytic
solution only; none of the method's code.

Set-up: a plane gap (phi = 0 at z = 0, phi = V at z = L, Neumann on x and y) whose lower
half holds a neutral plasma: one electron of weight w on the centre of every cell with
k < nz/2 and w positive ions in the same cell, D = 0.  With the TSC shape, electrons
and ions on the same centres spread alike, so the charge stays zero; the conductivity
of the lower layer spreads along z as 1 (the wall cell keeps the part that would fall
outside), ..., 1, 7/8, 1/8, 0, ..., and stays uniform over each x-y plane (the side
walls fold the same way).  The field of the 1-D operator with harmonic-mean faces is
then that of resistors in series: one flux through every face, phi rising by
flux x (face length / face coefficient).  Each electron sits on a centre and moves with
the TSC average (1/8, 3/4, 1/8 along z, folded at the walls) of E^{k+1}."""
import numpy as np

from semi_implicit_case import E_CHARGE, EPS0


def make_layer(base, shape="tsc", nz=24, grid_xy=(6, 5), eps_jump=1.5, L=1e-3, V=9e3, dt=0.5e-12):
    nx, ny = grid_xy
    dx = L / nz
    cfg = dict(base)
    cfg.update(name="layer", grid=(nx, ny, nz), dx=dx, V_anode=V, field="poisson", dt=dt, n_ppc=0,
               shape=shape, coeffs=dict(base["coeffs"], D=0.0, kgamma_ratio=0.0))
    co = cfg["coeffs"]
    mu = co["mu_a"] * (max(V / L, co["E_floor"]) / co["mu_E0"]) ** co["mu_b"]
    dV = dx ** 3
    w = int(round(eps_jump * EPS0 * dV / (E_CHARGE * mu * dt)))
    k, j, i = np.meshgrid(np.arange(nz // 2), np.arange(ny), np.arange(nx), indexing="ij")
    xi = np.stack([i.ravel(), j.ravel(), k.ravel()], axis=1) + 0.5
    cell = (i + nx * (j + ny * k)).ravel().astype(np.uint32)
    ids = np.arange(1, len(cell) + 1, dtype=np.uint64) * np.uint64(131)
    plus = np.zeros(nx * ny * nz, dtype=np.int64)
    plus[cell] = w
    # closed form (TSC profile)
    s = np.zeros(nz)
    s[: nz // 2] = 1.0
    s[nz // 2 - 1] = 0.875
    s[nz // 2] = 0.125
    sigma0 = E_CHARGE * mu * w / dV
    eps = 1.0 + sigma0 * s * dt / EPS0
    _, Ez = series_solution(eps, dx, V)
    kk = np.arange(nz)
    avg = 0.75 * Ez + 0.125 * Ez[np.maximum(kk - 1, 0)] + 0.125 * Ez[np.minimum(kk + 1, nz - 1)]
    dz = -mu * avg[(xi[:, 2] - 0.5).astype(int)] * dt / dx
    return dict(cfg=cfg, xi=xi, cell=cell, ids=ids, w=np.full(len(cell), w, dtype=np.uint64),
                nplus=plus, mu=mu, dx=dx, Ez_col=Ez, dz=dz)


def series_solution(eps, dx, V):
    """Cell-centred potential and central-difference E_z of the 1-D operator with
    harmonic-mean faces, phi = 0 below and V above (half-cell Dirichlet faces), zero
    charge."""
    faces = 2.0 * eps[:-1] * eps[1:] / (eps[:-1] + eps[1:])
    r = np.concatenate([[0.5 * dx / eps[0]], dx / faces, [0.5 * dx / eps[-1]]])
    flux = V / r.sum()
    phi = flux * np.cumsum(r)[:-1]
    ext = np.concatenate([[-phi[0]], phi, [2.0 * V - phi[-1]]])
    return phi, -(ext[2:] - ext[:-2]) / (2.0 * dx)
