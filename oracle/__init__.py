"""ctypes binding of the FP64 reference oracle (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``
may import this package.  The GPU library never loads it.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

FIELD_UNIFORM, FIELD_POISSON = 0, 1
KMC_HYBRID, KMC_PURE_TAU = 0, 1
SHAPES = {"cic": 0, "tsc": 1}
TAG_PUSH, TAG_SEED, TAG_KMC, TAG_CREATE, TAG_PHOTON = 1, 2, 3, 4, 5
KIND_SEED, KIND_KMC, KIND_PHOTO, KIND_MERGE = 0, 1, 2, 3


class Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("field_mode", ctypes.c_int32), ("dx", ctypes.c_double),
                ("E_uniform", ctypes.c_double * 3), ("V_anode", ctypes.c_double),
                ("kmc_mode", ctypes.c_int32), ("n_ppc", ctypes.c_int32),
                ("n_new", ctypes.c_int32), ("kmc_nc", ctypes.c_int32),
                ("kmc_nssa", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("kmc_eps", ctypes.c_double), ("seed", ctypes.c_uint32),
                ("realization", ctypes.c_uint32), ("poisson_rtol", ctypes.c_double)]


class Coeffs(ctypes.Structure):
    _fields_ = [("mu_a", ctypes.c_double), ("mu_E0", ctypes.c_double), ("mu_b", ctypes.c_double),
                ("E_floor", ctypes.c_double), ("D", ctypes.c_double),
                ("alpha_A", ctypes.c_double), ("alpha_B", ctypes.c_double),
                ("eta", ctypes.c_double), ("kgamma_ratio", ctypes.c_double),
                ("photon_l1", ctypes.c_double), ("photon_l2", ctypes.c_double),
                ("beta_ep", ctypes.c_double), ("beta_ep_b", ctypes.c_double),
                ("Te_a", ctypes.c_double), ("Te_b", ctypes.c_double),
                ("beta_np", ctypes.c_double), ("mu_ion", ctypes.c_double),
                ("D_ion", ctypes.c_double)]

# recombination coefficients are optional in a coefficient set (absent: reaction off),
# and so are the ion transport coefficients (absent: immobile ions)
RECOMB_FIELDS = ("beta_ep", "beta_ep_b", "Te_a", "Te_b", "beta_np")
ION_FIELDS = ("mu_ion", "D_ion")
OPTIONAL_FIELDS = RECOMB_FIELDS + ION_FIELDS


class Diag(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_uint64), ("weight", ctypes.c_uint64),
                ("n_plus", ctypes.c_int64), ("n_minus", ctypes.c_int64),
                ("charge", ctypes.c_int64), ("outflow_weight", ctypes.c_uint64),
                ("fires", ctypes.c_uint64 * 5), ("photons_emitted", ctypes.c_uint64),
                ("photons_absorbed", ctypes.c_uint64), ("photons_lost", ctypes.c_uint64),
                ("created", ctypes.c_uint64), ("removed_weight", ctypes.c_uint64),
                ("merged_cells", ctypes.c_uint64), ("step", ctypes.c_uint32),
                ("solver_iters", ctypes.c_int32), ("solver_relres", ctypes.c_double),
                ("ion_outflow_plus", ctypes.c_uint64), ("ion_outflow_minus", ctypes.c_uint64)]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if name == "fires" else v
        return out


class DtRule(ctypes.Structure):
    _fields_ = [("dt_max", ctypes.c_double), ("c_drift", ctypes.c_double),
                ("c_diff", ctypes.c_double), ("c_ion", ctypes.c_double)]


def make_dt_rule(rule) -> DtRule:
    """rule: dict with dt_max and any of c_drift, c_diff, c_ion (absent = off)."""
    return DtRule(float(rule["dt_max"]), float(rule.get("c_drift", 0.0)),
                  float(rule.get("c_diff", 0.0)), float(rule.get("c_ion", 0.0)))


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIBPATH)
        P = ctypes.c_void_p
        L.or_create.restype = P
        L.or_create.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Coeffs), ctypes.c_uint64]
        L.or_destroy.argtypes = [P]
        L.or_seed_gaussian.argtypes = [P, ctypes.c_uint64, P, ctypes.c_double]
        L.or_seed_neutral.argtypes = [P, ctypes.c_double, P, ctypes.c_double]
        L.or_set_particles.argtypes = [P, ctypes.c_uint64, P, P, P]
        L.or_num_particles.restype = ctypes.c_uint64
        L.or_num_particles.argtypes = [P]
        L.or_get_particles.argtypes = [P, P, P, P]
        L.or_set_counts.argtypes = [P, ctypes.c_int, P]
        L.or_get_counts.argtypes = [P, ctypes.c_int, P]
        L.or_set_step.argtypes = [P, ctypes.c_uint32]
        L.or_transport.argtypes = [P, ctypes.c_double]
        L.or_react.argtypes = [P, ctypes.c_double]
        L.or_step.argtypes = [P, ctypes.c_double, ctypes.c_uint32]
        L.or_diagnostics.argtypes = [P, ctypes.POINTER(Diag)]
        L.or_ngp_weight.argtypes = [P, P]
        L.or_cic_density.argtypes = [P, P]
        L.or_charge_density.argtypes = [P, P]
        L.or_poisson_relres.restype = ctypes.c_double
        L.or_poisson_relres.argtypes = [ctypes.POINTER(Desc), P, P, P]
        L.or_semi_implicit_residual.restype = ctypes.c_double
        L.or_semi_implicit_residual.argtypes = [P, ctypes.c_double, P]
        L.or_push_with_fields.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Coeffs),
                                          ctypes.c_uint64, P, P, ctypes.c_uint32,
                                          ctypes.c_double] + [P] * 7
        L.or_get_fires.argtypes = [P, P]
        L.or_get_field.argtypes = [P, P, P, P, P]
        L.or_set_field.argtypes = [P, P]
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_normals3.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                  ctypes.c_uint32, P]
        L.or_poisson_draw.restype = ctypes.c_int64
        L.or_poisson_draw.argtypes = [ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32,
                                      ctypes.c_uint32, ctypes.c_uint32, P]
        L.or_mobility.restype = ctypes.c_double
        L.or_mobility.argtypes = [ctypes.POINTER(Coeffs), ctypes.c_double]
        L.or_rates.argtypes = [ctypes.POINTER(Coeffs), ctypes.c_double, ctypes.c_double, P]
        L.or_kmc_leap_bound.argtypes = [ctypes.POINTER(Desc), P, P]
        L.or_kmc_leap_bound.restype = ctypes.c_double
        L.or_kmc_cells.argtypes = [ctypes.POINTER(Desc), ctypes.c_int64, P, P, P,
                                   ctypes.c_double, ctypes.c_uint32, P]
        L.or_merge_cell.restype = ctypes.c_int32
        L.or_merge_cell.argtypes = [ctypes.c_int32, ctypes.c_int32, P, P, P, ctypes.c_uint32,
                                    ctypes.c_uint32, P, P, P]
        L.or_solve_poisson.restype = ctypes.c_int
        L.or_solve_poisson.argtypes = [ctypes.POINTER(Desc), P, P, P, ctypes.c_double,
                                       ctypes.c_int, P]
        L.or_efield.argtypes = [ctypes.POINTER(Desc), P, P, P, P]
        L.or_cic_deposit.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint64, P, P, P]
        L.or_cic_interp.argtypes = [ctypes.POINTER(Desc), P, ctypes.c_uint64, P, P]
        L.or_tsc_deposit.argtypes = [ctypes.POINTER(Desc), ctypes.c_uint64, P, P, P]
        L.or_tsc_interp.argtypes = [ctypes.POINTER(Desc), P, ctypes.c_uint64, P, P]
        L.or_photons_cell.restype = ctypes.c_int32
        L.or_photons_cell.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Coeffs),
                                      ctypes.c_uint32, ctypes.c_int64, ctypes.c_uint32,
                                      P, P, P, P]
        L.or_field_max.restype = ctypes.c_double
        L.or_field_max.argtypes = [P]
        L.or_stable_dt.restype = ctypes.c_double
        L.or_stable_dt.argtypes = [P, ctypes.POINTER(DtRule), P]
        L.or_step_adaptive.argtypes = [P, ctypes.POINTER(DtRule), ctypes.c_uint32, P]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(cfg) -> Desc:
    """Build the oracle descriptor from a plain workload dict."""
    d = Desc()
    d.nx, d.ny, d.nz = cfg["grid"]
    d.dx = cfg["dx"]
    d.field_mode = FIELD_POISSON if cfg.get("field") == "poisson" else FIELD_UNIFORM
    d.E_uniform = (ctypes.c_double * 3)(*cfg.get("E", (0.0, 0.0, 0.0)))
    d.V_anode = cfg.get("V_anode", 0.0)
    d.kmc_mode = KMC_PURE_TAU if cfg.get("kmc") == "pure_tau" else KMC_HYBRID
    d.n_ppc = cfg.get("n_ppc", 0)
    d.n_new = cfg.get("n_new", 64)
    d.kmc_nc = cfg.get("kmc_nc", 5)
    d.kmc_nssa = cfg.get("kmc_nssa", 10)
    d.kmc_eps = cfg.get("kmc_eps", math.inf)
    d.seed = cfg.get("seed", 1)
    d.realization = cfg.get("realization", 0)
    d.poisson_rtol = cfg.get("oracle_rtol", 1e-13)
    d.shape = SHAPES[cfg.get("shape", "cic")]
    return d


def make_coeffs(cfg) -> Coeffs:
    c = Coeffs()
    co = cfg["coeffs"]
    for name, _ in Coeffs._fields_:
        setattr(c, name, co.get(name, 0.0) if name in OPTIONAL_FIELDS else co[name])
    return c


def philox(ctr, key):
    L = lib()
    c = np.asarray(ctr, dtype=np.uint32)
    k = np.asarray(key, dtype=np.uint32)
    o = np.zeros(4, dtype=np.uint32)
    L.or_philox4x32_10(_p(c), _p(k), _p(o))
    return o


def philox_many(ctrs, key):
    ctrs = np.ascontiguousarray(ctrs, dtype=np.uint32)
    out = np.zeros_like(ctrs)
    k = np.asarray(key, dtype=np.uint32)
    L = lib()
    for i in range(ctrs.shape[0]):
        L.or_philox4x32_10(_p(ctrs[i]), _p(k), _p(out[i]))
    return out


def normals3(pid, step, seed, realization):
    o = np.zeros(3)
    lib().or_normals3(int(pid), step, seed, realization, _p(o))
    return o


def poisson_draw(lam, cell, step, seed=1, realization=0):
    used = np.zeros(1, dtype=np.uint32)
    k = lib().or_poisson_draw(float(lam), cell, step, seed, realization, _p(used))
    return k, int(used[0])


def mobility(cfg, E):
    c = make_coeffs(cfg)
    return lib().or_mobility(ctypes.byref(c), float(E))


def rates(cfg, E):
    """(k_alpha, k_eta, k_gamma, k_ep, k_np) at field magnitude E in one cell of cfg."""
    c = make_coeffs(cfg)
    k = np.zeros(5)
    lib().or_rates(ctypes.byref(c), float(E), float(cfg["dx"]) ** 3, _p(k))
    return k


def _rates5(k, n):
    k = np.asarray(k, dtype=np.float64).reshape(n, -1)
    out = np.zeros((n, 5))
    out[:, :k.shape[1]] = k
    return out


def kmc_cells(cfg, X, k, dt, step, cell_ids=None):
    """One KMC step on independent cells. X: (n,4) int64, k: (n,3) or (n,5) (missing
    recombination rates are zero). Returns (X, fires (n,5))."""
    d = make_desc(cfg)
    X = np.ascontiguousarray(X, dtype=np.int64).copy()
    n = X.shape[0]
    k = np.ascontiguousarray(_rates5(k, n))
    if cell_ids is None:
        cell_ids = np.arange(n, dtype=np.uint32)
    cell_ids = np.ascontiguousarray(cell_ids, dtype=np.uint32)
    f = np.zeros((n, 5), dtype=np.int64)
    lib().or_kmc_cells(ctypes.byref(d), n, _p(cell_ids), _p(X), _p(k), float(dt), step, _p(f))
    return X, f


def kmc_leap_bound(cfg, X, k):
    """Step 4's non-critical leap bound for one state X (4) and rates k (3 or 5)."""
    d = make_desc(cfg)
    X = np.ascontiguousarray(X, dtype=np.int64)
    k = np.ascontiguousarray(_rates5(k, 1)[0])
    return lib().or_kmc_leap_bound(ctypes.byref(d), _p(X), _p(k))


def merge_cell(n_ppc, off, w, ids, cell=0, step=0):
    off = np.ascontiguousarray(off, dtype=np.float64)
    w = np.ascontiguousarray(w, dtype=np.uint64)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    m = w.shape[0]
    oo = np.zeros((max(n_ppc, 1), 3))
    ow = np.zeros(max(n_ppc, 1), dtype=np.uint64)
    oi = np.zeros(max(n_ppc, 1), dtype=np.uint64)
    nl = lib().or_merge_cell(n_ppc, m, _p(off), _p(w), _p(ids), cell, step, _p(oo), _p(ow), _p(oi))
    return oo[:nl], ow[:nl], oi[:nl]


def solve_poisson(cfg, rho, eps_r, phi0=None, rtol=1e-13, max_iter=200000):
    d = make_desc(cfg)
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    eps_r = np.ascontiguousarray(eps_r, dtype=np.float64)
    phi = np.zeros_like(rho) if phi0 is None else np.ascontiguousarray(phi0, dtype=np.float64).copy()
    rr = np.zeros(1)
    it = lib().or_solve_poisson(ctypes.byref(d), _p(rho), _p(eps_r), _p(phi), rtol, max_iter, _p(rr))
    return phi, it, float(rr[0])


def efield(cfg, phi):
    d = make_desc(cfg)
    phi = np.ascontiguousarray(phi, dtype=np.float64)
    E = [np.zeros_like(phi) for _ in range(3)]
    lib().or_efield(ctypes.byref(d), _p(phi), _p(E[0]), _p(E[1]), _p(E[2]))
    return E


def cic_deposit(cfg, xi, q):
    d = make_desc(cfg)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    nx, ny, nz = cfg["grid"]
    g = np.zeros(nx * ny * nz)
    lib().or_cic_deposit(ctypes.byref(d), q.shape[0], _p(xi), _p(q), _p(g))
    return g


def cic_interp(cfg, grid, xi):
    d = make_desc(cfg)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    out = np.zeros(xi.shape[0])
    lib().or_cic_interp(ctypes.byref(d), _p(grid), xi.shape[0], _p(xi), _p(out))
    return out


def tsc_deposit(cfg, xi, q):
    d = make_desc(cfg)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    q = np.ascontiguousarray(q, dtype=np.float64)
    nx, ny, nz = cfg["grid"]
    g = np.zeros(nx * ny * nz)
    lib().or_tsc_deposit(ctypes.byref(d), q.shape[0], _p(xi), _p(q), _p(g))
    return g


def tsc_interp(cfg, grid, xi):
    d = make_desc(cfg)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    grid = np.ascontiguousarray(grid, dtype=np.float64)
    out = np.zeros(xi.shape[0])
    lib().or_tsc_interp(ctypes.byref(d), _p(grid), xi.shape[0], _p(xi), _p(out))
    return out


def cloud_interp(cfg, grid, xi):
    """Interpolation with cfg's particle shape (CIC unless cfg['shape'] == 'tsc')."""
    return tsc_interp(cfg, grid, xi) if cfg.get("shape", "cic") == "tsc" else cic_interp(cfg, grid, xi)


def photons_cell(cfg, cell, n_gamma, step):
    d = make_desc(cfg)
    c = make_coeffs(cfg)
    cap = max(d.n_new, 1)
    xi = np.zeros((cap, 3))
    w = np.zeros(cap, dtype=np.uint64)
    ids = np.zeros(cap, dtype=np.uint64)
    lost = np.zeros(1, dtype=np.uint64)
    n = lib().or_photons_cell(ctypes.byref(d), ctypes.byref(c), cell, int(n_gamma), step,
                              _p(xi), _p(w), _p(ids), _p(lost))
    return xi[:n], w[:n], ids[:n], int(lost[0])


class Sim:
    """One oracle realization (positions in grid units)."""

    def __init__(self, cfg, capacity=0):
        self.cfg = cfg
        self._d = make_desc(cfg)
        self._c = make_coeffs(cfg)
        self.ncell = int(np.prod(cfg["grid"]))
        self.h = lib().or_create(ctypes.byref(self._d), ctypes.byref(self._c), capacity)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_destroy(self.h)
            self.h = None

    def seed_gaussian(self, n0, centre, sigma):
        c = np.asarray(centre, dtype=np.float64)
        return lib().or_seed_gaussian(self.h, n0, _p(c), sigma)

    def seed_neutral(self, n_peak, centre, sigma):
        c = np.asarray(centre, dtype=np.float64)
        return lib().or_seed_neutral(self.h, n_peak, _p(c), sigma)

    def set_particles(self, xi, w, ids):
        xi = np.ascontiguousarray(xi, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.uint64)
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        lib().or_set_particles(self.h, w.shape[0], _p(xi), _p(w), _p(ids))

    def particles(self):
        n = lib().or_num_particles(self.h)
        xi = np.zeros((n, 3))
        w = np.zeros(n, dtype=np.uint64)
        ids = np.zeros(n, dtype=np.uint64)
        lib().or_get_particles(self.h, _p(xi), _p(w), _p(ids))
        return xi, w, ids

    def counts(self, which):
        v = np.zeros(self.ncell, dtype=np.int64)
        lib().or_get_counts(self.h, {"plus": 0, "minus": 1, "gamma": 2}[which], _p(v))
        return v

    def set_counts(self, which, v):
        v = np.ascontiguousarray(v, dtype=np.int64)
        lib().or_set_counts(self.h, {"plus": 0, "minus": 1, "gamma": 2}[which], _p(v))

    def set_step(self, k):
        lib().or_set_step(self.h, k)

    def transport(self, dt):
        return lib().or_transport(self.h, dt)

    def react(self, dt):
        return lib().or_react(self.h, dt)

    def step(self, dt, n=1):
        return lib().or_step(self.h, dt, n)

    def diagnostics(self):
        dg = Diag()
        lib().or_diagnostics(self.h, ctypes.byref(dg))
        return dg.as_dict()

    def field_max(self):
        return float(lib().or_field_max(self.h))

    def stable_dt(self, rule):
        """(dt, Emax) of the dynamic time-step rule for the next step."""
        r = make_dt_rule(rule)
        em = np.zeros(1)
        dt = lib().or_stable_dt(self.h, ctypes.byref(r), _p(em))
        return float(dt), float(em[0])

    def step_adaptive(self, rule, n):
        r = make_dt_rule(rule)
        dts = np.zeros(max(int(n), 1))
        rc = lib().or_step_adaptive(self.h, ctypes.byref(r), int(n), _p(dts))
        if rc:
            raise RuntimeError("oracle adaptive step failed")
        return dts[:int(n)]

    def ngp_weight(self):
        v = np.zeros(self.ncell, dtype=np.int64)
        lib().or_ngp_weight(self.h, _p(v))
        return v

    def cic_density(self):
        v = np.zeros(self.ncell)
        lib().or_cic_density(self.h, _p(v))
        return v

    def charge_density(self):
        v = np.zeros(self.ncell)
        lib().or_charge_density(self.h, _p(v))
        return v

    def semi_implicit_residual(self, dt, phi):
        """||b - A phi|| / ||b|| in the system this state's transport would solve."""
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        return lib().or_semi_implicit_residual(self.h, float(dt), _p(phi))

    def fires(self):
        v = np.zeros((self.ncell, 3), dtype=np.int64)
        lib().or_get_fires(self.h, _p(v))
        return v

    def field(self):
        out = [np.zeros(self.ncell) for _ in range(4)]
        lib().or_get_field(self.h, *[_p(a) for a in out])
        return out

    def set_field(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        lib().or_set_field(self.h, _p(phi))

    def set_efield(self, Ex, Ey, Ez):
        E = [np.ascontiguousarray(a, dtype=np.float64) for a in (Ex, Ey, Ez)]
        L = lib()
        L.or_set_efield.argtypes = [ctypes.c_void_p] * 4
        L.or_set_efield(self.h, *[_p(a) for a in E])


def photon_sample(cfg, cell, slot, step):
    d = make_desc(cfg)
    c = make_coeffs(cfg)
    y0 = np.zeros(3)
    dr = np.zeros(3)
    r = np.zeros(1)
    L = lib()
    L.or_photon_sample.argtypes = [ctypes.POINTER(Desc), ctypes.POINTER(Coeffs), ctypes.c_uint32,
                                   ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_void_p]
    L.or_photon_sample(ctypes.byref(d), ctypes.byref(c), cell, slot, step, _p(y0), _p(dr), _p(r))
    return y0, dr, float(r[0])


def poisson_relres(cfg, rho, eps_r, phi):
    d = make_desc(cfg)
    a = [np.ascontiguousarray(x, dtype=np.float64) for x in (rho, eps_r, phi)]
    return lib().or_poisson_relres(ctypes.byref(d), *[_p(x) for x in a])


def push_with_fields(cfg, xi, ids, step, dt, Ek, Ek1):
    """Semi-implicit update of particles xi (grid units) with given cell-centred fields
    Ek = (Ex, Ey, Ez) at step k and Ek1 at step k+1."""
    d = make_desc(cfg)
    c = make_coeffs(cfg)
    xi = np.ascontiguousarray(xi, dtype=np.float64)
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    F = [np.ascontiguousarray(a, dtype=np.float64) for a in list(Ek) + list(Ek1)]
    out = np.zeros_like(xi)
    lib().or_push_with_fields(ctypes.byref(d), ctypes.byref(c), xi.shape[0], _p(xi), _p(ids),
                              step, float(dt), *[_p(a) for a in F], _p(out))
    return out
