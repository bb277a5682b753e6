"""Seeded synthetic workloads (plain data; none of the method's arithmetic lives here).

Each preset is a plain dict consumed both by the GPU library binding and by the
test oracle.  The transport and rate data are synthetic air-like stand-ins for the
BOLSIG+/SIGLO tables the paper uses (which are not available):
    mu(E) = 0.0372 (E / 1e6 V/m)^-0.25 m^2/(V s),  D = 0.1 m^2/s,
    alpha(E) = 4.332e5 exp(-1.91e7 / E) 1/m,        eta = 2000 1/m,
    k_gamma = 0.06 k_alpha (photo-emission, self-consistent presets only),
    photon absorption length log-uniform in [30 um, 2 mm].
Random parameters of ensemble presets are drawn here with numpy's generator; they
are inputs, not part of the method.
"""
import copy
import math

import numpy as np

AIR = dict(mu_a=0.0372, mu_E0=1.0e6, mu_b=-0.25, E_floor=1.0e4, D=0.1,
           alpha_A=4.332e5, alpha_B=1.91e7, eta=2000.0, kgamma_ratio=0.0,
           photon_l1=30e-6, photon_l2=2e-3)

# Recombination rows of the air chemistry, with the paper's rate coefficients
# beta_ep = 1.138e-11 T_e^-0.7 m^3/s and beta_np = 2e-13 m^3/s (gas at 300 K) and a
# synthetic electron temperature T_e = max(300 K, 1e4 K (E / 1 MV/m)^0.5) (about 2.7 eV
# at 10 MV/m) in place of the tabulated T_e(E).  Off in every preset above unless merged
# in (coefficients absent count as zero).
RECOMBINATION = dict(beta_ep=1.138e-11, beta_ep_b=-0.7, Te_a=1.0e4, Te_b=0.5, beta_np=2.0e-13)

# Plain avalanche: 32^3 grid, dx = 10 um, uniform 10 MV/m along z, 1e4 electrons of
# weight 1 in a Gaussian blob (sigma = 50 um) at the centre, dt = 1 ps, 200 steps,
# NGP deposit, hybrid KMC for ionization and attachment, seed 1, FP64.
AVALANCHE_32 = dict(
    name="avalanche_32", grid=(32, 32, 32), dx=10e-6, field="uniform", E=(0.0, 0.0, 1.0e7),
    coeffs=dict(AIR), kmc="hybrid", n_ppc=0, n_new=64, seed=1, realization=0,
    precision="fp64", dt=1e-12, steps=200,
    seed_kind="gaussian", seed_n0=10000, seed_centre=(160e-6, 160e-6, 160e-6), seed_sigma=50e-6,
)

# Self-consistent positive streamer: 1 mm plane-plane gap, 256^3 cells, 18 kV on
# z = L, neutral Gaussian plasma seed (sigma = 40 um, peak 1e20 m^-3) centred
# 100 um below the anode, semi-implicit Poisson each step, photo-emission at 0.06 x
# ionization, merge/split to 32 particles per cell, FP32 particle state, dt = 0.5 ps.
STREAMER_256 = dict(
    name="streamer_256", grid=(256, 256, 256), dx=1e-3 / 256, field="poisson", V_anode=18e3,
    coeffs=dict(AIR, kgamma_ratio=0.06), kmc="hybrid", n_ppc=32, n_new=64, seed=1,
    realization=0, precision="fp32", dt=0.5e-12, steps=4000, max_particles=50_000_000,
    seed_kind="neutral", seed_peak=1e20, seed_centre=(0.5e-3, 0.5e-3, 0.9e-3), seed_sigma=40e-6,
    gmg_rtol=1e-10,
)

# The same streamer at the particle cap: a denser, wider seed (peak 1e21 m^-3,
# sigma = 65 um) at the centre of the gap makes about 7.7e7 computational particles
# (at most 64 per cell), and the first superparticle pass leaves about 4.4e7 (32 per
# cell where the count allows).  The bank holds the seed and, before that first pass,
# the reactions' products (up to 64 per cell): 1.6e8 slots.
STREAMER_256_DENSE = dict(STREAMER_256, name="streamer_256_dense", seed_peak=1e21,
                          seed_centre=(0.5e-3, 0.5e-3, 0.5e-3), seed_sigma=65e-6,
                          max_particles=160_000_000)

# The 256^3 streamer with the quadratic B-spline (TSC) shape for the conductivity and
# charge deposits and the field interpolation (27 cells per particle instead of 8).
STREAMER_256_TSC = dict(STREAMER_256, name="streamer_256_tsc", shape="tsc")

# The 256^3 streamer with mobile ions: ion mobility 2e-4 m^2/(V s) (of the order of
# atmospheric-pressure N2+/O2- mobilities) and the Einstein diffusion coefficient at 300 K,
# mu_ion k T / e = 5.2e-6 m^2/s.
IONS = dict(mu_ion=2e-4, D_ion=5.2e-6)
STREAMER_256_IONS = dict(STREAMER_256, name="streamer_256_ions", coeffs=dict(STREAMER_256["coeffs"], **IONS))

# The same gap at 64^3 (dx = 15.6 um), 200 steps: precision study size.
STREAMER_64 = dict(STREAMER_256, name="streamer_64", grid=(64, 64, 64), dx=1e-3 / 64,
                   steps=200, max_particles=4_000_000)


# Avalanche at streamer scale: the plain-method physics of AVALANCHE_32 on the
# streamer's 256^3 grid (dx = 3.9 um), 5e7 weight-1 electrons in a Gaussian blob
# (sigma = 150 um), FP32 state.  Exercises push, binning, NGP deposit, KMC and coupling
# at the particle count of the self-consistent workload.
AVALANCHE_256 = dict(
    AVALANCHE_32, name="avalanche_256", grid=(256, 256, 256), dx=1e-3 / 256,
    precision="fp32", seed_n0=50_000_000, seed_centre=(0.5e-3, 0.5e-3, 0.5e-3),
    seed_sigma=150e-6, max_particles=110_000_000, steps=40,
)


# Zero-dimensional reactors (the paper's comparison of the reaction algorithm with the
# rate equation): electron-impact ionization and attachment only, no transport, the
# synthetic air coefficients at a fixed field.  After the paper's two cases: (a) above
# breakdown, E = 10 MV/m, one starting electron, 50 ps (50 steps of 1 ps); (b) below
# breakdown, E = 1.7 MV/m, five starting electrons, 50 ns (500 steps of 100 ps).  A
# reactor ensemble holds n_reactors independent reactors (stream cell ids 0 .. n-1) at
# the field magnitude E_field (V/m).
REACTOR_A = dict(name="reactor_a", kind="reactor", coeffs=dict(AIR), kmc="hybrid", seed=1,
                 realization=0, E_field=1.0e7, X0=1, n_reactors=1_000_000, dt=1e-12, steps=50,
                 dx=10e-6, grid=(8, 8, 8), field="uniform", precision="fp64")
REACTOR_B = dict(REACTOR_A, name="reactor_b", E_field=1.7e6, X0=5, n_reactors=200_000, dt=1e-10,
                 steps=500)


def preset(name, **overrides):
    base = {"avalanche_32": AVALANCHE_32, "streamer_256": STREAMER_256,
            "streamer_64": STREAMER_64, "avalanche_256": AVALANCHE_256,
            "streamer_256_dense": STREAMER_256_DENSE, "streamer_256_tsc": STREAMER_256_TSC,
            "streamer_256_ions": STREAMER_256_IONS,
            "reactor_a": REACTOR_A,
            "reactor_b": REACTOR_B}[name]
    cfg = copy.deepcopy(base)
    for k, v in overrides.items():
        if k == "coeffs":
            cfg["coeffs"].update(v)
        else:
            cfg[k] = v
    return cfg


def ensemble_realization(r, seed=1):
    """Batched-avalanche realization r: grid edge uniform in {32, 48, 64, 96} (dx = 5 um),
    initial electrons log-uniform in [1e3, 1e5], uniform field log-uniform in
    [3, 12] MV/m, 500 steps of 1 ps or until 1e6 particles, FP32 state.  A realization
    stops after the first step that began with at least stop_particles live particles;
    its particle quota (max_particles) leaves room for that step's growth.  Parameters
    are drawn from a generator keyed by (seed, r), so realization r is the same in any
    batch or request stream."""
    rng = np.random.default_rng([seed, r])
    edge = int(rng.choice([32, 48, 64, 96]))
    n0 = int(round(10 ** rng.uniform(3, 5)))
    E = float(10 ** rng.uniform(math.log10(3e6), math.log10(1.2e7)))
    L = edge * 5e-6
    return dict(
        name=f"ens_{r}", grid=(edge, edge, edge), dx=5e-6, field="uniform", E=(0.0, 0.0, E),
        coeffs=dict(AIR), kmc="hybrid", n_ppc=0, n_new=64, seed=seed, realization=r,
        precision="fp32", dt=1e-12, steps=500, stop_particles=1_000_000,
        max_particles=1_250_000,
        seed_kind="gaussian", seed_n0=n0, seed_centre=(L / 2, L / 2, L / 2),
        seed_sigma=0.156 * L)


def ensemble_realizations(n=256, seed=1):
    """The first n batched-avalanche realizations (see ensemble_realization)."""
    return [ensemble_realization(r, seed) for r in range(n)]


def poisson_request(r, seed=1):
    """Self-consistent served request r: 128^3 grid, dx = 5 um (L = 640 um), plane
    electrodes at V = E L with E drawn as for the batched avalanches, the same Gaussian
    electron seed, semi-implicit Poisson each step, no photons or merging, 500 steps of
    1 ps or until 1e6 particles, FP32 state."""
    rng = np.random.default_rng([seed, r, 128])
    n0 = int(round(10 ** rng.uniform(3, 5)))
    E = float(10 ** rng.uniform(math.log10(3e6), math.log10(1.2e7)))
    L = 128 * 5e-6
    return dict(
        name=f"poisson_{r}", grid=(128, 128, 128), dx=5e-6, field="poisson", V_anode=E * L,
        coeffs=dict(AIR), kmc="hybrid", n_ppc=0, n_new=64, seed=seed, realization=r,
        precision="fp32", dt=1e-12, steps=500, stop_particles=1_000_000,
        max_particles=1_250_000, gmg_rtol=1e-10,
        seed_kind="gaussian", seed_n0=n0, seed_centre=(L / 2, L / 2, L / 2),
        seed_sigma=0.156 * L)


def reactor_request(r, seed=1):
    """Served zero-dimensional request r: an ensemble of 4096 reactors (as REACTOR_A) with
    the field log-uniform in [1.7, 12] MV/m, the starting electrons log-uniform in
    [1, 100] and 50 to 500 steps of 1 ps; the key (seed, r)."""
    rng = np.random.default_rng([seed, r, 0])
    E = float(10 ** rng.uniform(math.log10(1.7e6), math.log10(1.2e7)))
    X0 = int(round(10 ** rng.uniform(0, 2)))
    steps = int(rng.integers(50, 501))
    return dict(REACTOR_A, coeffs=dict(AIR), name=f"reactor_{r}", E_field=E, X0=X0,
                n_reactors=4096, steps=steps, seed=seed, realization=r)


def request_trace(rate=200.0, duration=60.0, poisson_frac=0.1, seed=1, reactor_frac=0.0):
    """Served workload: Poisson arrivals at `rate` requests/s over `duration` s; each
    request is a self-consistent 128^3 request with probability poisson_frac, a
    zero-dimensional reactor ensemble with probability reactor_frac, else a
    batched-avalanche realization.  Returns [(arrival_s, request_id, cfg)]."""
    rng = np.random.default_rng([seed, 5])
    out = []
    t = 0.0
    r = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return out
        u = rng.random()
        if u < poisson_frac:
            cfg = poisson_request(r, seed)
        elif reactor_frac > 0.0 and u < poisson_frac + reactor_frac:
            cfg = reactor_request(r, seed)
        else:
            cfg = ensemble_realization(r, seed)
        out.append((t, r, cfg))
        r += 1


def random_particles(rng, grid, n, wmax=1, id_base=0):
    """Uniform random particles in grid units with integer weights in [1, wmax] and
    distinct ids (for unit-level parity tests)."""
    g = np.asarray(grid, dtype=np.float64)
    xi = rng.random((n, 3)) * g
    w = rng.integers(1, wmax + 1, size=n).astype(np.uint64)
    ids = (np.uint64(id_base) + rng.permutation(np.arange(n, dtype=np.uint64) * np.uint64(7) + np.uint64(3)))
    return xi, w, ids
