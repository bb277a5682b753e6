"""Python binding of libitokmc (the C ABI in include/itokmc.h).

Argument marshalling only: every step of the method runs in the HIP kernels of the
library.  PyTorch supplies the device arena and the stream.  Importing this module on
a machine without the built library raises immediately; there is no fallback.
"""
import ctypes
import math
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libitokmc.so")

OK, EINVAL, ENOMEM, ECAPACITY, ENOCONV, EHIP, EAGAIN = 0, -1, -2, -3, -4, -5, -6
SLOT_FREE, SLOT_ACTIVE, SLOT_DONE, SLOT_CAPPED = 0, 1, 2, 3
FP32, FP64 = 0, 1
FIELD_UNIFORM, FIELD_POISSON = 0, 1
KMC_HYBRID, KMC_PURE_TAU = 0, 1
SEED_GAUSSIAN, SEED_NEUTRAL = 0, 1
(Q_NGP_WEIGHT, Q_NPLUS, Q_NMINUS, Q_NGAMMA, Q_CIC_DENSITY, Q_PHI, Q_EX, Q_EY, Q_EZ, Q_FIRES,
 Q_RHO) = range(11)
OVF_PARTICLES, OVF_MERGE, OVF_BARRIER = 1, 2, 4

EXPORTS = ["itokmc_arena_bytes", "itokmc_init_grid", "itokmc_set_coefficients",
           "itokmc_check_coefficients",
           "itokmc_seed_particles", "itokmc_step", "itokmc_transport", "itokmc_react",
           "itokmc_deposit", "itokmc_diagnostics", "itokmc_get_particles",
           "itokmc_set_particles", "itokmc_get_counts", "itokmc_set_counts", "itokmc_set_step",
           "itokmc_get_field", "itokmc_set_field", "itokmc_destroy", "itokmc_last_error",
           "itokmc_philox_fill", "itokmc_kmc_cells", "itokmc_kmc_run", "itokmc_rates",
           "itokmc_step_until", "itokmc_stable_dt", "itokmc_step_adaptive",
           "itokmc_set_profiling",
           "itokmc_phase_times", "itokmc_set_tuning", "itokmc_get_tuning",
           "itokmc_ensemble_arena_bytes", "itokmc_ensemble_create", "itokmc_ensemble_admit",
           "itokmc_ensemble_step", "itokmc_ensemble_poll", "itokmc_ensemble_result",
           "itokmc_ensemble_results",
           "itokmc_ensemble_get_particles", "itokmc_ensemble_get_counts",
           "itokmc_ensemble_release", "itokmc_ensemble_info", "itokmc_ensemble_set_tuning",
           "itokmc_ensemble_get_tuning", "itokmc_ensemble_autotune", "itokmc_ensemble_destroy",
           "itokmc_ensemble_last_error", "itokmc_sort_workspace_bytes", "itokmc_sort_by_cell",
           "itokmc_sort_by_cell_noalloc"]
SHAPES = {"cic": 0, "tsc": 1}
PHASES = ["push", "photons", "scan", "scatter", "kmc", "couple", "deposit", "solve",
          "field_push", "count", "merge", "field_prep", "smooth_fine", "couple_light", "emax",
          "ions"]


class GridDesc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("dx", ctypes.c_double),
                ("field_mode", ctypes.c_int32), ("kmc_mode", ctypes.c_int32),
                ("E_uniform", ctypes.c_double * 3), ("V_anode", ctypes.c_double),
                ("n_ppc", ctypes.c_int32), ("n_new", ctypes.c_int32),
                ("kmc_nc", ctypes.c_int32), ("kmc_nssa", ctypes.c_int32),
                ("kmc_eps", ctypes.c_double), ("seed", ctypes.c_uint32),
                ("realization", ctypes.c_uint32), ("max_particles", ctypes.c_uint64),
                ("gmg_max_cycles", ctypes.c_int32), ("shape", ctypes.c_int32),
                ("gmg_rtol", ctypes.c_double)]


class DtRule(ctypes.Structure):
    _fields_ = [("dt_max", ctypes.c_double), ("c_drift", ctypes.c_double),
                ("c_diff", ctypes.c_double), ("c_ion", ctypes.c_double)]


def make_dt_rule(rule) -> DtRule:
    """rule: dict with dt_max and any of c_drift, c_diff, c_ion (absent = off)."""
    return DtRule(float(rule["dt_max"]), float(rule.get("c_drift", 0.0)),
                  float(rule.get("c_diff", 0.0)), float(rule.get("c_ion", 0.0)))


class Coeffs(ctypes.Structure):
    _fields_ = [(n, ctypes.c_double) for n in ("mu_a", "mu_E0", "mu_b", "E_floor", "D", "alpha_A",
                                               "alpha_B", "eta", "kgamma_ratio", "photon_l1",
                                               "photon_l2", "beta_ep", "beta_ep_b", "Te_a", "Te_b",
                                               "beta_np", "mu_ion", "D_ion")]


# recombination coefficients are optional in a coefficient set (absent: reaction off)
RECOMB_FIELDS = ("beta_ep", "beta_ep_b", "Te_a", "Te_b", "beta_np")
ION_FIELDS = ("mu_ion", "D_ion")
OPTIONAL_FIELDS = RECOMB_FIELDS + ION_FIELDS


class Tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("mg_pre", "mg_post", "bottom_sweeps", "use_graph",
                                              "extrapolate", "fine_layout")]


class SeedDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("pad0", ctypes.c_int32), ("n0", ctypes.c_uint64),
                ("centre", ctypes.c_double * 3), ("sigma", ctypes.c_double),
                ("n_peak", ctypes.c_double)]


class Diag(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_uint64), ("weight", ctypes.c_uint64),
                ("n_plus", ctypes.c_int64), ("n_minus", ctypes.c_int64),
                ("charge", ctypes.c_int64), ("outflow_weight", ctypes.c_uint64),
                ("fires", ctypes.c_uint64 * 5), ("photons_emitted", ctypes.c_uint64),
                ("photons_absorbed", ctypes.c_uint64), ("photons_lost", ctypes.c_uint64),
                ("created", ctypes.c_uint64), ("removed_weight", ctypes.c_uint64),
                ("merged_cells", ctypes.c_uint64), ("step", ctypes.c_uint32),
                ("solver_cycles", ctypes.c_int32), ("solver_relres", ctypes.c_double),
                ("rho_sum", ctypes.c_double), ("overflow", ctypes.c_uint32),
                ("occupied_cells", ctypes.c_uint32), ("particle_steps", ctypes.c_uint64),
                ("merge_skipped", ctypes.c_uint32), ("queued_cells", ctypes.c_uint32),
                ("solver_cycles_total", ctypes.c_uint64), ("solves_total", ctypes.c_uint64),
                ("couple_pieces", ctypes.c_uint64), ("wave_cells", ctypes.c_uint32),
                ("pad2", ctypes.c_uint32), ("ion_outflow_plus", ctypes.c_uint64),
                ("ion_outflow_minus", ctypes.c_uint64)]

    def as_dict(self):
        d = {}
        for n, _ in self._fields_:
            if n.startswith("pad"):
                continue
            v = getattr(self, n)
            d[n] = list(v) if n == "fires" else v
        return d


class EnsDesc(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_cells", ctypes.c_uint64), ("max_particles", ctypes.c_uint64)]


class RunDesc(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_double), ("nsteps", ctypes.c_uint32), ("pad0", ctypes.c_uint32),
                ("stop_particles", ctypes.c_uint64), ("tag", ctypes.c_uint64)]


class SlotEvent(ctypes.Structure):
    _fields_ = [("slot", ctypes.c_int32), ("state", ctypes.c_int32), ("tag", ctypes.c_uint64),
                ("steps", ctypes.c_uint32), ("pad0", ctypes.c_uint32)]


class EnsInfo(ctypes.Structure):
    _fields_ = [("slots_used", ctypes.c_int32), ("slots_free", ctypes.c_int32),
                ("cells_free", ctypes.c_uint64), ("particles_free", ctypes.c_uint64),
                ("pool_particles", ctypes.c_uint64), ("steps", ctypes.c_uint64)]


class EnsTuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("push_block", "push_blocks_per_cu", "kmc_block",
                                              "couple_per_cu", "use_graph", "fused_per_cu")]


class ItokmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"itokmc error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    """Load libitokmc.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is missing: run __graft_entry__.build() first")
        L = ctypes.CDLL(LIBPATH)
        P, U32, U64, I32, D = (ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int,
                               ctypes.c_double)
        L.itokmc_arena_bytes.restype = ctypes.c_size_t
        L.itokmc_arena_bytes.argtypes = [ctypes.POINTER(GridDesc)]
        L.itokmc_init_grid.argtypes = [ctypes.POINTER(P), ctypes.POINTER(GridDesc), P,
                                       ctypes.c_size_t, P]
        L.itokmc_set_coefficients.argtypes = [P, ctypes.POINTER(Coeffs)]
        L.itokmc_check_coefficients.argtypes = [ctypes.POINTER(Coeffs)]
        L.itokmc_seed_particles.argtypes = [P, ctypes.POINTER(SeedDesc)]
        L.itokmc_step.argtypes = [P, U32, D]
        L.itokmc_step_until.argtypes = [P, U32, D, U64, P]
        L.itokmc_stable_dt.argtypes = [P, ctypes.POINTER(DtRule), P]
        L.itokmc_step_adaptive.argtypes = [P, ctypes.POINTER(DtRule), U32, P]
        L.itokmc_transport.argtypes = [P, D]
        L.itokmc_react.argtypes = [P, D]
        L.itokmc_deposit.argtypes = [P, I32, P]
        L.itokmc_diagnostics.argtypes = [P, ctypes.POINTER(Diag)]
        L.itokmc_get_particles.argtypes = [P, ctypes.POINTER(U64), P, P, P, P]
        L.itokmc_set_particles.argtypes = [P, U64, P, P, P, P]
        L.itokmc_get_counts.argtypes = [P, I32, P]
        L.itokmc_set_counts.argtypes = [P, I32, P]
        L.itokmc_set_step.argtypes = [P, U32]
        L.itokmc_get_field.argtypes = [P, P]
        L.itokmc_set_field.argtypes = [P, P]
        L.itokmc_destroy.argtypes = [P]
        L.itokmc_destroy.restype = None
        L.itokmc_last_error.argtypes = [P]
        L.itokmc_last_error.restype = ctypes.c_char_p
        L.itokmc_philox_fill.argtypes = [U32, U32, U32, U32, U32, U32, U64, P, P]
        L.itokmc_kmc_cells.argtypes = [P, U64, P, P, P, D, U32, P]
        L.itokmc_kmc_run.argtypes = [P, U64, P, P, P, P, P, D, U32, U32, P]
        L.itokmc_rates.argtypes = [ctypes.POINTER(Coeffs), D, D, P]
        L.itokmc_set_profiling.argtypes = [P, I32]
        L.itokmc_set_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.itokmc_get_tuning.argtypes = [P, ctypes.POINTER(Tuning)]
        L.itokmc_phase_times.argtypes = [P, P, P, I32, I32]
        L.itokmc_ensemble_arena_bytes.restype = ctypes.c_size_t
        L.itokmc_ensemble_arena_bytes.argtypes = [ctypes.POINTER(EnsDesc)]
        L.itokmc_ensemble_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(EnsDesc), P,
                                             ctypes.c_size_t, P]
        L.itokmc_ensemble_admit.argtypes = [P, ctypes.POINTER(GridDesc), ctypes.POINTER(Coeffs),
                                            ctypes.POINTER(SeedDesc), ctypes.POINTER(RunDesc),
                                            ctypes.POINTER(ctypes.c_int32)]
        L.itokmc_ensemble_step.argtypes = [P, U32]
        L.itokmc_ensemble_poll.argtypes = [P, P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]
        L.itokmc_ensemble_result.argtypes = [P, ctypes.c_int32, ctypes.POINTER(Diag)]
        L.itokmc_ensemble_results.argtypes = [P, P, ctypes.c_int32, P]
        L.itokmc_ensemble_get_particles.argtypes = [P, ctypes.c_int32, ctypes.POINTER(U64), P, P,
                                                    P, P]
        L.itokmc_ensemble_get_counts.argtypes = [P, ctypes.c_int32, I32, P]
        L.itokmc_ensemble_release.argtypes = [P, ctypes.c_int32]
        L.itokmc_ensemble_info.argtypes = [P, ctypes.POINTER(EnsInfo)]
        L.itokmc_ensemble_set_tuning.argtypes = [P, ctypes.POINTER(EnsTuning)]
        L.itokmc_ensemble_get_tuning.argtypes = [P, ctypes.POINTER(EnsTuning)]
        L.itokmc_ensemble_autotune.argtypes = [P, U32, ctypes.POINTER(EnsTuning),
                                               ctypes.POINTER(ctypes.c_double)]
        L.itokmc_ensemble_destroy.argtypes = [P]
        L.itokmc_ensemble_destroy.restype = None
        L.itokmc_ensemble_last_error.argtypes = [P]
        L.itokmc_ensemble_last_error.restype = ctypes.c_char_p
        L.itokmc_sort_workspace_bytes.restype = ctypes.c_size_t
        L.itokmc_sort_workspace_bytes.argtypes = [U64, U32]
        L.itokmc_sort_by_cell.argtypes = [I32, U64, U32] + [P] * 14 + [P, ctypes.c_size_t, P]
        L.itokmc_sort_by_cell_noalloc.argtypes = [I32, U64, U32] + [P] * 14 + [P]
        _lib = L
    return _lib


def _np(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def make_desc(cfg, precision=None, max_particles=None):
    d = GridDesc()
    d.nx, d.ny, d.nz = cfg["grid"]
    prec = precision or cfg.get("precision", "fp32")
    d.precision = FP64 if prec == "fp64" else FP32
    d.dx = cfg["dx"]
    d.field_mode = FIELD_POISSON if cfg.get("field") == "poisson" else FIELD_UNIFORM
    d.kmc_mode = KMC_PURE_TAU if cfg.get("kmc") == "pure_tau" else KMC_HYBRID
    d.E_uniform = (ctypes.c_double * 3)(*cfg.get("E", (0.0, 0.0, 0.0)))
    d.V_anode = cfg.get("V_anode", 0.0)
    d.n_ppc = cfg.get("n_ppc", 0)
    d.n_new = cfg.get("n_new", 64)
    d.kmc_nc = cfg.get("kmc_nc", 5)
    d.kmc_nssa = cfg.get("kmc_nssa", 10)
    d.kmc_eps = cfg.get("kmc_eps", math.inf)
    d.seed = cfg.get("seed", 1)
    d.realization = cfg.get("realization", 0)
    d.max_particles = int(max_particles or cfg.get("max_particles", 4_000_000))
    d.gmg_max_cycles = cfg.get("gmg_max_cycles", 50)
    d.gmg_rtol = cfg.get("gmg_rtol", 1e-10)
    d.shape = SHAPES[cfg.get("shape", "cic")]
    return d


def arena_bytes(cfg, precision=None, max_particles=None):
    """Device bytes a single context for cfg needs (0 if the descriptor is invalid)."""
    return lib().itokmc_arena_bytes(ctypes.byref(make_desc(cfg, precision, max_particles)))


def make_coeffs(cfg):
    c = Coeffs()
    for n, _ in Coeffs._fields_:
        setattr(c, n, cfg["coeffs"].get(n, 0.0) if n in OPTIONAL_FIELDS else cfg["coeffs"][n])
    return c


class Sim:
    """One realization resident on a GPU."""

    def __init__(self, cfg, device="cuda:0", precision=None, max_particles=None, stream=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lib()
        self._desc = make_desc(cfg, precision, max_particles)
        nbytes = L.itokmc_arena_bytes(ctypes.byref(self._desc))
        if nbytes == 0:
            raise ItokmcError(EINVAL, "invalid grid descriptor")
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.ncell = int(np.prod(cfg["grid"]))
        h = ctypes.c_void_p()
        rc = L.itokmc_init_grid(ctypes.byref(h), ctypes.byref(self._desc),
                                ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                                ctypes.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise ItokmcError(rc, "init_grid failed")
        self.h = h
        self._check(L.itokmc_set_coefficients(self.h, ctypes.byref(make_coeffs(cfg))))

    def _check(self, rc):
        if rc != OK:
            msg = lib().itokmc_last_error(self.h).decode()
            raise ItokmcError(rc, msg)
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().itokmc_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- setup ---------------------------------------------------------------------
    def seed(self):
        return self._check(lib().itokmc_seed_particles(self.h, ctypes.byref(make_seed(self.cfg))))

    # -- stepping ------------------------------------------------------------------
    def step(self, n=1, dt=None):
        return self._check(lib().itokmc_step(self.h, n, dt or self.cfg["dt"]))

    def stable_dt(self, rule):
        """(dt, Emax) of the dynamic time-step rule for the next step (synchronises)."""
        r = make_dt_rule(rule)
        out = np.zeros(2)
        self._check(lib().itokmc_stable_dt(self.h, ctypes.byref(r), _np(out)))
        return float(out[0]), float(out[1])

    def step_adaptive(self, rule, n):
        """n steps, each of the rule's dt at its start; returns the dts."""
        r = make_dt_rule(rule)
        dts = np.zeros(max(int(n), 1))
        self._check(lib().itokmc_step_adaptive(self.h, ctypes.byref(r), int(n), _np(dts)))
        return dts[:int(n)]

    def step_until(self, n, stop_particles=0, dt=None):
        """Up to n steps under the device-side stop rule; returns the number of steps
        taken (prescribed-field mode: one synchronisation; self-consistent mode: the
        host reads the rule's decision after each step)."""
        done = ctypes.c_uint32(0)
        self._check(lib().itokmc_step_until(self.h, n, dt or self.cfg["dt"], int(stop_particles),
                                             ctypes.byref(done)))
        return done.value

    def step_rc(self, n=1, dt=None):
        return lib().itokmc_step(self.h, n, dt or self.cfg["dt"])

    def transport(self, dt=None):
        return self._check(lib().itokmc_transport(self.h, dt or self.cfg["dt"]))

    def react(self, dt=None):
        return self._check(lib().itokmc_react(self.h, dt or self.cfg["dt"]))

    def set_step(self, k):
        return self._check(lib().itokmc_set_step(self.h, k))

    # -- queries -------------------------------------------------------------------
    def diagnostics(self, check=True):
        d = Diag()
        rc = lib().itokmc_diagnostics(self.h, ctypes.byref(d))
        if check:
            self._check(rc)
        return d.as_dict()

    def particles(self):
        n = ctypes.c_uint64()
        self._check(lib().itokmc_get_particles(self.h, ctypes.byref(n), None, None, None, None))
        N = n.value
        cell = np.zeros(N, dtype=np.uint32)
        off = np.zeros((N, 3), dtype=np.float64)
        w = np.zeros(N, dtype=np.uint32)
        ids = np.zeros(N, dtype=np.uint64)
        self._check(lib().itokmc_get_particles(self.h, ctypes.byref(n), _np(cell), _np(off), _np(w),
                                               _np(ids)))
        assert n.value == N
        return cell, off, w, ids

    def set_particles(self, cell, off, w, ids):
        cell = np.ascontiguousarray(cell, dtype=np.uint32)
        off = np.ascontiguousarray(off, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.uint32)
        ids = np.ascontiguousarray(ids, dtype=np.uint64)
        return self._check(lib().itokmc_set_particles(self.h, len(w), _np(cell), _np(off), _np(w),
                                                      _np(ids)))

    def counts(self, which):
        q = {"plus": Q_NPLUS, "minus": Q_NMINUS, "gamma": Q_NGAMMA}[which]
        v = np.zeros(self.ncell, dtype=np.uint32)
        self._check(lib().itokmc_get_counts(self.h, q, _np(v)))
        return v

    def set_counts(self, which, v):
        q = {"plus": Q_NPLUS, "minus": Q_NMINUS, "gamma": Q_NGAMMA}[which]
        v = np.ascontiguousarray(v, dtype=np.uint32)
        return self._check(lib().itokmc_set_counts(self.h, q, _np(v)))

    def deposit(self, what):
        torch = self.torch
        q = {"ngp": Q_NGP_WEIGHT, "plus": Q_NPLUS, "minus": Q_NMINUS, "gamma": Q_NGAMMA,
             "cic": Q_CIC_DENSITY, "phi": Q_PHI, "ex": Q_EX, "ey": Q_EY, "ez": Q_EZ,
             "fires": Q_FIRES, "rho": Q_RHO}[what]
        if q in (Q_CIC_DENSITY, Q_PHI, Q_EX, Q_EY, Q_EZ, Q_RHO):
            out = torch.empty(self.ncell, dtype=torch.float64, device=self.device)
        elif q == Q_FIRES:
            out = torch.empty(self.ncell * 3, dtype=torch.int32, device=self.device)
        else:
            out = torch.empty(self.ncell, dtype=torch.int32, device=self.device)
        self._check(lib().itokmc_deposit(self.h, q, ctypes.c_void_p(out.data_ptr())))
        self.stream.synchronize()
        a = out.cpu().numpy()
        if q == Q_FIRES:
            return a.view(np.uint32).reshape(self.ncell, 3)
        if a.dtype == np.int32:
            return a.view(np.uint32)
        return a

    def tuning(self):
        t = Tuning()
        self._check(lib().itokmc_get_tuning(self.h, ctypes.byref(t)))
        return {n: getattr(t, n) for n, _ in Tuning._fields_}

    def set_tuning(self, **kw):
        t = Tuning()
        self._check(lib().itokmc_get_tuning(self.h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        return self._check(lib().itokmc_set_tuning(self.h, ctypes.byref(t)))

    def set_profiling(self, on):
        return self._check(lib().itokmc_set_profiling(self.h, 1 if on else 0))

    def phase_times(self, reset=True):
        """{phase: (total ms, launches)} from HIP events on the library's stream."""
        n = len(PHASES)
        ms = np.zeros(n)
        calls = np.zeros(n, dtype=np.uint64)
        self._check(lib().itokmc_phase_times(self.h, _np(ms), _np(calls), n, 1 if reset else 0))
        return {p: (float(ms[i]), int(calls[i])) for i, p in enumerate(PHASES)}

    def field(self):
        phi = np.zeros(self.ncell)
        self._check(lib().itokmc_get_field(self.h, _np(phi)))
        return phi

    def set_field(self, phi):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        return self._check(lib().itokmc_set_field(self.h, _np(phi)))

    def kmc_cells(self, X, k, dt, step, cell_ids=None):
        """One KMC step on independent cells (kernel-level entry point).  k: (n,3) or
        (n,5) rates (missing recombination rates are zero); returns X and fires (n,5)."""
        torch = self.torch
        X = np.ascontiguousarray(X, dtype=np.int64)
        n = X.shape[0]
        ids = np.arange(n, dtype=np.uint32) if cell_ids is None else np.asarray(cell_ids, np.uint32)
        k = np.asarray(k, dtype=np.float64).reshape(n, -1)
        k5 = np.zeros((n, 5))
        k5[:, :k.shape[1]] = k
        dX = torch.from_numpy(X.copy()).to(self.device)
        dk = torch.from_numpy(k5).to(self.device)
        di = torch.from_numpy(ids.astype(np.int32)).to(self.device)
        df = torch.zeros((n, 5), dtype=torch.int64, device=self.device)
        self.stream.synchronize()
        self._check(lib().itokmc_kmc_cells(self.h, n, ctypes.c_void_p(di.data_ptr()),
                                           ctypes.c_void_p(dX.data_ptr()),
                                           ctypes.c_void_p(dk.data_ptr()), dt, step,
                                           ctypes.c_void_p(df.data_ptr())))
        self.stream.synchronize()
        return dX.cpu().numpy(), df.cpu().numpy()


    def kmc_run_device(self, ids, X, k, dt, step0, nsteps, fires, realization=None,
                       steps=None):
        """Zero-dimensional reactors on device tensors (kernel-level entry point):
        ids (n,) int32, X (n,4) int64 in/out, k (n,5) float64, fires (n,5) int64 out,
        realization and steps (n,) int32 or None.  Enqueued on the context's stream."""
        n = X.shape[0]
        rp = ctypes.c_void_p(realization.data_ptr()) if realization is not None else None
        sp = ctypes.c_void_p(steps.data_ptr()) if steps is not None else None
        return self._check(lib().itokmc_kmc_run(self.h, n, ctypes.c_void_p(ids.data_ptr()), rp, sp,
                                                ctypes.c_void_p(X.data_ptr()),
                                                ctypes.c_void_p(k.data_ptr()), dt, step0, nsteps,
                                                ctypes.c_void_p(fires.data_ptr())))

    def kmc_run(self, X, k, dt, step0, nsteps, cell_ids=None, realization=None):
        """Host-array form of kmc_run_device; returns X and the fire totals (n,5)."""
        torch = self.torch
        X = np.ascontiguousarray(X, dtype=np.int64)
        n = X.shape[0]
        ids = np.arange(n, dtype=np.uint32) if cell_ids is None else np.asarray(cell_ids, np.uint32)
        k = np.asarray(k, dtype=np.float64).reshape(n, -1)
        k5 = np.zeros((n, 5))
        k5[:, :k.shape[1]] = k
        dX = torch.from_numpy(X.copy()).to(self.device)
        dk = torch.from_numpy(k5).to(self.device)
        di = torch.from_numpy(ids.astype(np.int32)).to(self.device)
        dr = None
        if realization is not None:
            dr = torch.from_numpy(np.asarray(realization, np.uint32).astype(np.int32)).to(self.device)
        df = torch.zeros((n, 5), dtype=torch.int64, device=self.device)
        self.stream.synchronize()
        self.kmc_run_device(di, dX, dk, dt, step0, nsteps, df, dr)
        self.stream.synchronize()
        return dX.cpu().numpy(), df.cpu().numpy()


def rates(cfg, E):
    """The library's rate constants (k_alpha, k_eta, k_gamma, k_ep, k_np) in 1/s at field
    magnitude E in one cell of cfg (host computation, no device)."""
    out = (ctypes.c_double * 5)()
    rc = lib().itokmc_rates(ctypes.byref(make_coeffs(cfg)), float(E), float(cfg["dx"]), out)
    if rc != OK:
        raise ItokmcError(rc, "invalid coefficients or field")
    return np.array(list(out))


def make_seed(cfg):
    sd = SeedDesc()
    sd.centre = (ctypes.c_double * 3)(*cfg["seed_centre"])
    sd.sigma = cfg["seed_sigma"]
    if cfg["seed_kind"] == "gaussian":
        sd.kind = SEED_GAUSSIAN
        sd.n0 = cfg["seed_n0"]
    else:
        sd.kind = SEED_NEUTRAL
        sd.n_peak = cfg["seed_peak"]
    return sd


def make_run(cfg, tag=0):
    r = RunDesc()
    r.dt = cfg["dt"]
    r.nsteps = int(cfg["steps"])
    r.stop_particles = int(cfg.get("stop_particles", 0))
    r.tag = int(tag)
    return r


class Ensemble:
    """Many independent uniform-field realizations advanced together on one GPU
    (the itokmc_ensemble_* entry points)."""

    def __init__(self, max_slots, max_cells, max_particles, precision="fp32", device="cuda:0",
                 stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        L = lib()
        self._desc = EnsDesc(int(max_slots), FP64 if precision == "fp64" else FP32,
                             int(max_cells), int(max_particles))
        nbytes = L.itokmc_ensemble_arena_bytes(ctypes.byref(self._desc))
        if nbytes == 0:
            raise ItokmcError(EINVAL, "invalid ensemble descriptor")
        self.arena_bytes = nbytes
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        rc = L.itokmc_ensemble_create(ctypes.byref(h), ctypes.byref(self._desc),
                                      ctypes.c_void_p(self.arena.data_ptr()), nbytes,
                                      ctypes.c_void_p(self.stream.cuda_stream))
        if rc != OK:
            raise ItokmcError(rc, "ensemble_create failed")
        self.h = h
        self.ncell = {}
        self.max_slots = int(max_slots)
        self._ev = (SlotEvent * self.max_slots)()

    @staticmethod
    def arena_bytes_for(max_slots, max_cells, max_particles, precision="fp32"):
        d = EnsDesc(int(max_slots), FP64 if precision == "fp64" else FP32, int(max_cells),
                    int(max_particles))
        return lib().itokmc_ensemble_arena_bytes(ctypes.byref(d))

    def _check(self, rc):
        if rc != OK:
            raise ItokmcError(rc, lib().itokmc_ensemble_last_error(self.h).decode())
        return rc

    def close(self):
        if getattr(self, "h", None):
            lib().itokmc_ensemble_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def admit(self, cfg, tag=0):
        """Admit one realization; returns its slot, or None if the pools are full."""
        slot = ctypes.c_int32(-1)
        rc = lib().itokmc_ensemble_admit(self.h, ctypes.byref(make_desc(cfg)),
                                         ctypes.byref(make_coeffs(cfg)),
                                         ctypes.byref(make_seed(cfg)),
                                         ctypes.byref(make_run(cfg, tag)), ctypes.byref(slot))
        if rc == EAGAIN:
            return None
        self._check(rc)
        self.ncell[slot.value] = int(np.prod(cfg["grid"]))
        return slot.value

    def step(self, n=1):
        return self._check(lib().itokmc_ensemble_step(self.h, n))

    def poll(self):
        """[(slot, state, tag, steps)] of realizations finished since the last poll."""
        out = []
        while True:
            n = ctypes.c_int32()
            self._check(lib().itokmc_ensemble_poll(self.h, self._ev, self.max_slots,
                                                   ctypes.byref(n)))
            out += [(e.slot, e.state, e.tag, e.steps) for e in self._ev[:n.value]]
            if n.value < self.max_slots:
                return out

    def result(self, slot):
        d = Diag()
        self._check(lib().itokmc_ensemble_result(self.h, slot, ctypes.byref(d)))
        return d.as_dict()

    def results(self, slots):
        """Diagnostics of several resident realizations with one pass over the pool."""
        slots = list(slots)
        if not slots:
            return []
        arr = (ctypes.c_int32 * len(slots))(*slots)
        out = (Diag * len(slots))()
        self._check(lib().itokmc_ensemble_results(self.h, ctypes.cast(arr, ctypes.c_void_p),
                                                  len(slots), ctypes.cast(out, ctypes.c_void_p)))
        return [d.as_dict() for d in out]

    def particles(self, slot):
        n = ctypes.c_uint64()
        self._check(lib().itokmc_ensemble_get_particles(self.h, slot, ctypes.byref(n), None, None,
                                                        None, None))
        N = n.value
        cell = np.zeros(N, dtype=np.uint32)
        off = np.zeros((N, 3), dtype=np.float64)
        w = np.zeros(N, dtype=np.uint32)
        ids = np.zeros(N, dtype=np.uint64)
        self._check(lib().itokmc_ensemble_get_particles(self.h, slot, ctypes.byref(n), _np(cell),
                                                        _np(off), _np(w), _np(ids)))
        return cell, off, w, ids

    def counts(self, slot, which):
        q = {"ngp": Q_NGP_WEIGHT, "plus": Q_NPLUS, "minus": Q_NMINUS}[which]
        v = np.zeros(self.ncell[slot], dtype=np.uint32)
        self._check(lib().itokmc_ensemble_get_counts(self.h, slot, q, _np(v)))
        return v

    def release(self, slot):
        self.ncell.pop(slot, None)
        return self._check(lib().itokmc_ensemble_release(self.h, slot))

    def info(self):
        i = EnsInfo()
        self._check(lib().itokmc_ensemble_info(self.h, ctypes.byref(i)))
        return {n: getattr(i, n) for n, _ in EnsInfo._fields_}

    def tuning(self):
        t = EnsTuning()
        self._check(lib().itokmc_ensemble_get_tuning(self.h, ctypes.byref(t)))
        return {n: getattr(t, n) for n, _ in EnsTuning._fields_}

    def set_tuning(self, **kw):
        t = EnsTuning()
        self._check(lib().itokmc_ensemble_get_tuning(self.h, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        return self._check(lib().itokmc_ensemble_set_tuning(self.h, ctypes.byref(t)))

    def autotune(self, rounds=3):
        t = EnsTuning()
        ms = ctypes.c_double()
        self._check(lib().itokmc_ensemble_autotune(self.h, rounds, ctypes.byref(t),
                                                   ctypes.byref(ms)))
        return {n: getattr(t, n) for n, _ in EnsTuning._fields_}, ms.value


def philox_fill(c0, c1, c2, c3, k0, k1, n, device="cuda:0"):
    import torch
    out = torch.empty(4 * n, dtype=torch.int32, device=device)
    rc = lib().itokmc_philox_fill(c0, c1, c2, c3, k0, k1, n, ctypes.c_void_p(out.data_ptr()),
                                  ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream))
    if rc != OK:
        raise ItokmcError(rc, "philox_fill")
    torch.cuda.synchronize(device)
    return out.cpu().numpy().view(np.uint32).reshape(n, 4)


def _sort_tensors(cell, off, w, ids, precision, device):
    import torch
    ft = torch.float64 if precision == "fp64" else torch.float32
    dev = torch.device(device)
    t = {"cell": torch.from_numpy(np.ascontiguousarray(cell, dtype=np.uint32).view(np.int32)).to(dev),
         "w": torch.from_numpy(np.ascontiguousarray(w, dtype=np.uint32).view(np.int32)).to(dev),
         "id": torch.from_numpy(np.ascontiguousarray(ids, dtype=np.uint64).view(np.int64)).to(dev)}
    off = np.asarray(off, dtype=np.float64).reshape(-1, 3)
    for a, k in enumerate(("ox", "oy", "oz")):
        t[k] = torch.from_numpy(np.ascontiguousarray(off[:, a])).to(dev, ft)
    return t


def sort_by_cell(cell, off, w, ids, ncell, precision="fp32", device="cuda:0", noalloc=False):
    """Counting sort of particles by cell through the C ABI (kernel-level entry point).
    Returns (start[ncell+1], cell, off (n, 3), w, ids) of the live particles, grouped by
    cell, as numpy arrays."""
    import torch
    L = lib()
    n = len(w)
    t = _sort_tensors(cell, off, w, ids, precision, device)
    o = {k: torch.empty_like(v) for k, v in t.items()}
    start = torch.empty(ncell + 1, dtype=torch.int32, device=device)
    n_out = torch.zeros(1, dtype=torch.int32, device=device)
    stream = torch.cuda.current_stream(torch.device(device))
    prec = FP64 if precision == "fp64" else FP32
    args = [prec, n, ncell] + [ctypes.c_void_p(t[k].data_ptr()) for k in ("cell", "ox", "oy", "oz", "w", "id")] + \
        [ctypes.c_void_p(o[k].data_ptr()) for k in ("cell", "ox", "oy", "oz", "w", "id")] + \
        [ctypes.c_void_p(start.data_ptr()), ctypes.c_void_p(n_out.data_ptr())]
    if noalloc:
        rc = L.itokmc_sort_by_cell_noalloc(*args, ctypes.c_void_p(stream.cuda_stream))
    else:
        nb = L.itokmc_sort_workspace_bytes(n, ncell)
        ws = torch.empty(max(nb, 1), dtype=torch.uint8, device=device)
        rc = L.itokmc_sort_by_cell(*args, ctypes.c_void_p(ws.data_ptr()), nb,
                                   ctypes.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise ItokmcError(rc, "sort_by_cell failed")
    stream.synchronize()
    m = int(n_out.cpu().item())
    offs = np.stack([o[k][:m].double().cpu().numpy() for k in ("ox", "oy", "oz")], axis=1)
    return (start.cpu().numpy().view(np.uint32), o["cell"][:m].cpu().numpy().view(np.uint32), offs,
            o["w"][:m].cpu().numpy().view(np.uint32), o["id"][:m].cpu().numpy().view(np.uint64))
