/*
 * itokmc -- MI355X (gfx950) library for one time step of the Ito-KMC particle-mesh
 * method of Marskar, "Stochastic and self-consistent 3D modeling of streamer
 * discharge trees with Kinetic Monte Carlo": the Ito drift-diffusion push of
 * computational electrons (eq. ito_kernel), field interpolation and NGP/CIC
 * deposition (section "Charge deposition & interpolation"), binning of particles by
 * cell, per-cell Kinetic Monte Carlo (section "Kinetic Monte Carlo" and its
 * "Reaction algorithm outline"), the KMC-particle coupling of eq. w, photon
 * transport (eq. photon_transport), superparticle merge/split (section
 * "Superparticle management", eq. weight_median) and the semi-implicit field solve
 * (eqs. poisson_simp and conductivity) on a uniform Cartesian grid with planar
 * electrodes at z = 0 (grounded) and z = L, in the step order of the paper's "Final
 * algorithm".
 *
 * Conventions for every entry point:
 *   - Return value: ITOKMC_OK (0) or a negative ITOKMC_E* code; nothing throws or
 *     aborts across this boundary.  itokmc_last_error() gives a message.
 *   - Device work is enqueued on the stream given to itokmc_init_grid (a hipStream_t
 *     passed as void*).  Calls that return host data synchronise that stream.
 *   - Memory: the caller allocates one device arena of itokmc_arena_bytes() bytes
 *     and keeps it alive until itokmc_destroy; the library sub-allocates all device
 *     buffers from it and never allocates device memory itself.  Host pointers are
 *     only read or written during the call.
 *   - Units are SI: m, s, V, V/m, m^-3.  Positions cross the boundary as cell index
 *     plus cell-relative offset in [0,1) per axis.
 *   - A context is not thread-safe; use one context per stream.
 *   - Cells are numbered c = i + nx (j + ny k); at most 2^24 cells.
 */
#ifndef ITOKMC_H
#define ITOKMC_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  ITOKMC_OK = 0,
  ITOKMC_EINVAL = -1,    /* invalid argument or descriptor                     */
  ITOKMC_ENOMEM = -2,    /* arena too small                                     */
  ITOKMC_ECAPACITY = -3, /* particle capacity exceeded; state stays valid      */
  ITOKMC_ENOCONV = -4,   /* field solve did not reach its tolerance            */
  ITOKMC_EHIP = -5,      /* a HIP runtime call failed                           */
  ITOKMC_EAGAIN = -6     /* ensemble: no free slot, cells or particle quota now  */
};
enum { ITOKMC_FP32 = 0, ITOKMC_FP64 = 1 };
enum { ITOKMC_FIELD_UNIFORM = 0, ITOKMC_FIELD_POISSON = 1 };
enum { ITOKMC_KMC_HYBRID = 0, ITOKMC_KMC_PURE_TAU = 1 };
/* Particle shape of the field coupling: the conductivity and charge deposits and the
 * field interpolation of the self-consistent mode, and the density and charge queries
 * in either mode, all use it.  CIC: the tent of the section
 * "Charge deposition & interpolation".  TSC: the quadratic B-spline (the tent averaged
 * over a unit box, 27 cells), one of the higher-order deposits of the section "Future
 * work"; along an axis with centres at j + 1/2, nearest centre j, offset d in
 * [-1/2, 1/2): weights (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2; a centre outside the
 * grid hands its weight to the wall cell; the immobile ions, point charges at their
 * cell centres, take the same shape. */
enum { ITOKMC_SHAPE_CIC = 0, ITOKMC_SHAPE_TSC = 1 };
enum { ITOKMC_SEED_GAUSSIAN = 0, ITOKMC_SEED_NEUTRAL = 1 };
/* itokmc_deposit / counts selectors */
enum {
  ITOKMC_Q_NGP_WEIGHT = 0, /* uint32 per cell: sum of electron weights (NGP)          */
  ITOKMC_Q_NPLUS = 1,      /* uint32 per cell: positive ions                          */
  ITOKMC_Q_NMINUS = 2,     /* uint32 per cell: negative ions                          */
  ITOKMC_Q_NGAMMA = 3,     /* uint32 per cell: photons pending transport              */
  ITOKMC_Q_CIC_DENSITY = 4,/* double per cell: electron density (m^-3) with the grid's
                              shape (CIC, or TSC when selected)                      */
  ITOKMC_Q_PHI = 5,        /* double per cell: potential (V), field mode POISSON      */
  ITOKMC_Q_EX = 6, ITOKMC_Q_EY = 7, ITOKMC_Q_EZ = 8, /* double per cell: E (V/m)     */
  ITOKMC_Q_FIRES = 9,      /* uint32 per cell x 3: ionization, attachment and emission
                              fires of the last step (recombination: totals only)    */
  ITOKMC_Q_RHO = 10        /* double per cell: space charge e((n+ - n-)/dV - n_e) with
                              n_e the density of the current particles and the ions
                              deposited with the grid's shape (C/m^3)                */
};
/* itokmc_diag.overflow flags (any set flag makes itokmc_diagnostics return ECAPACITY) */
enum {
  ITOKMC_OVF_PARTICLES = 1, /* a particle bank was full: particles that did not fit
                               were dropped                                         */
  ITOKMC_OVF_MERGE = 2,     /* a cell held more particles than the largest merge
                               staging (1536 in FP32, 1024 in FP64): it was left
                               unmerged (merge_skipped counts such cells)            */
  ITOKMC_OVF_BARRIER = 4    /* ensemble, fused step: a device-wide barrier gave up
                               waiting (its grid was not resident at once); that step
                               did not complete and the ensemble's state is not valid */
};

typedef struct itokmc_ctx itokmc_ctx;

/* Grid and method parameters (section "Computer implementation"; defaults are the
 * paper's: n_new = 64 (section "KMC-particle coupling"), kmc_nc = 5, kmc_nssa = 10,
 * kmc_eps = +inf (section "Final algorithm"), gmg_rtol = 1e-10). */
typedef struct {
  int32_t nx, ny, nz;
  int32_t precision;       /* ITOKMC_FP32: single-precision offsets and push,
                              ITOKMC_FP64: double everywhere                         */
  double dx;               /* cell edge (m)                                          */
  int32_t field_mode;      /* ITOKMC_FIELD_UNIFORM | ITOKMC_FIELD_POISSON            */
  int32_t kmc_mode;        /* ITOKMC_KMC_HYBRID | ITOKMC_KMC_PURE_TAU                */
  double E_uniform[3];     /* prescribed field (V/m), uniform mode                   */
  double V_anode;          /* potential of z = L (V), Poisson mode                   */
  int32_t n_ppc;           /* superparticle target per cell (<= 64); 0 = no merge    */
  int32_t n_new;           /* max computational particles made per cell and step     */
  int32_t kmc_nc;          /* critical-reaction threshold N_c                        */
  int32_t kmc_nssa;        /* max SSA events per SSA excursion                        */
  double kmc_eps;          /* leap accuracy factor; INFINITY accepts any leap        */
  uint32_t seed, realization; /* key of every random stream                          */
  uint64_t max_particles;  /* particle capacity (per bank)                           */
  int32_t gmg_max_cycles;  /* max multigrid cycles per solve                          */
  int32_t shape;           /* ITOKMC_SHAPE_CIC | ITOKMC_SHAPE_TSC                     */
  double gmg_rtol;         /* relative residual target of the field solve            */
} itokmc_grid_desc;

/* Transport and rate coefficients as functions of |E| (local field approximation,
 * section "Particle transport"): mu(E) = mu_a (max(E,E_floor)/mu_E0)^mu_b, constant
 * D, alpha(E) = alpha_A exp(-alpha_B/E), eta constant; k_alpha = alpha mu E,
 * k_eta = eta mu E, k_gamma = kgamma_ratio k_alpha; photon mean absorption length
 * log-uniform in [photon_l1, photon_l2].
 * Recombination (the electron-ion and ion-ion rows of the air-chemistry table, rates of
 * the section "Simulation conditions"; each reaction is off when its coefficient is 0):
 * k_ep = beta_ep T_e^beta_ep_b / dV with the electron temperature
 * T_e = max(300 K, Te_a (max(E,E_floor)/mu_E0)^Te_b) (a synthetic stand-in for the
 * tabulated T_e(E)), k_np = beta_np / dV; propensities k_ep X_e X_M+ and
 * k_np X_M+ X_M-.  The batched ensemble does not take recombination (EINVAL).
 * Ion transport (the paper moves ions as Ito particles and proposes heavy species as a
 * continuum in the section "Future work"): the ion counts stay per cell and move, once
 * per transport with the step's field E^{k+1} (the prescribed field in the uniform
 * mode), as a lattice jump process: an ion of sign q crosses the face towards its
 * neighbour along an axis in direction d = -1, +1 at the rate
 * max(0, d q mu_ion E_face) / dx + D_ion / dx^2 (E_face: mean of the two cell-centre
 * fields, the cell's own on a domain face); per step each face's count is
 * Poisson(n rate dt), n the count before the move, drawn for M+ then M- in the order
 * -x, +x, -y, +y, -z, +z, each from its own stream (cell, step, ION, sub = 6 species +
 * face), each capped at the ions not yet moved; ions leaving the domain are tallied in
 * itokmc_diag.  The batched
 * ensemble does not take mobile ions (EINVAL). */
typedef struct {
  double mu_a, mu_E0, mu_b, E_floor, D, alpha_A, alpha_B, eta, kgamma_ratio;
  double photon_l1, photon_l2;
  double beta_ep, beta_ep_b, Te_a, Te_b, beta_np;
  double mu_ion, D_ion;   /* ion transport (see below); both 0: immobile ions          */
} itokmc_coeffs;

/* Initial particles.  GAUSSIAN: n0 electrons of weight 1 at centre + sigma N(0,1)^3,
 * draws outside the domain discarded.  NEUTRAL: per cell Poisson(n_peak
 * exp(-r^2/2 sigma^2) dV) electron-ion pairs, electrons made by the coupling rule. */
typedef struct {
  int32_t kind;
  int32_t pad0;
  uint64_t n0;
  double centre[3];
  double sigma;
  double n_peak;
} itokmc_seed_desc;

typedef struct {
  uint64_t n_particles, weight;
  int64_t n_plus, n_minus;
  int64_t charge;                 /* sum(n+ - n_e - n-), units of e                  */
  uint64_t outflow_weight;
  uint64_t fires[5];              /* cumulative: ionization, attachment, emission,
                                     electron-ion and ion-ion recombination          */
  uint64_t photons_emitted, photons_absorbed, photons_lost;
  uint64_t created, removed_weight, merged_cells;
  uint32_t step;
  int32_t solver_cycles;          /* last field solve                                 */
  double solver_relres;
  double rho_sum;                 /* FP64 sum of rho dV over the grid (C)             */
  uint32_t overflow;              /* nonzero if a capacity limit was hit             */
  uint32_t occupied_cells;        /* cells holding particles at the last binning     */
  uint64_t particle_steps;        /* cumulative live particles advanced by transport */
  uint32_t merge_skipped;         /* cells whose particles exceeded the merge staging */
  uint32_t queued_cells;          /* cells coupled (and merged) by the last step      */
  uint64_t solver_cycles_total;   /* multigrid cycles over all field solves          */
  uint64_t solves_total;          /* field solves performed                           */
  uint64_t couple_pieces;         /* cumulative particles gathered by the wavefront
                                     coupling pass (cells with merging or many particles) */
  uint32_t wave_cells;            /* cells of the last step's wavefront coupling pass  */
  uint32_t pad2;
  uint64_t ion_outflow_plus;      /* cumulative positive and negative ions lost      */
  uint64_t ion_outflow_minus;     /* through domain faces (mobile ions)              */
} itokmc_diag;

/* Bytes of device arena needed for a descriptor (0 if the descriptor is invalid).
 * Host-only: no device call.  The arena holds two particle banks of max_particles
 * (structure of arrays), the per-cell arrays and, in POISSON mode, the multigrid
 * levels (section "Computer implementation"). */
size_t itokmc_arena_bytes(const itokmc_grid_desc* desc);

/* Create a context for one realization on a uniform grid with planar electrodes
 * (the paper's problem statement, eq. ito_poisson, on the grid of section "Computer
 * implementation").  arena: device pointer of at least itokmc_arena_bytes(desc)
 * bytes, 256-byte aligned, owned by the caller.  stream: hipStream_t (may be NULL).
 * The context starts with no particles, zero ion counts and step 0.
 * Errors: EINVAL (bad descriptor or null arena), ENOMEM (arena too small), EHIP. */
int itokmc_init_grid(itokmc_ctx** out, const itokmc_grid_desc* desc, void* arena,
                     size_t arena_bytes, void* stream);

/* Set the coefficient set (copied): the field-dependent mobility, diffusion and rate
 * coefficients of the local field approximation (section "Particle transport", the
 * rates k_r of section "Kinetic Monte Carlo") and the photon absorption lengths
 * (eq. photon_transport).  EINVAL on a non-finite or negative coefficient (the
 * previous set stays in force). */
int itokmc_set_coefficients(itokmc_ctx* ctx, const itokmc_coeffs* coeffs);
/* The same validation without a context (host-only, no device call): ITOKMC_OK or
 * ITOKMC_EINVAL. */
int itokmc_check_coefficients(const itokmc_coeffs* coeffs);
/* Rate constants (1/s) at field magnitude E (V/m) in a cell of edge dx (m), host-only:
 * out[5] = k_alpha = alpha mu E, k_eta = eta mu E, k_gamma = kgamma_ratio k_alpha (the
 * local field approximation of the section "Particle transport" and the air-chemistry
 * table), k_ep and k_np (section "Simulation conditions"; 0 when off).  EINVAL on
 * invalid coefficients, E < 0 or dx <= 0. */
int itokmc_rates(const itokmc_coeffs* coeffs, double E, double dx, double* out);

/* Seed particles (appends to the current state; step counter unchanged).  GAUSSIAN:
 * n0 weight-1 electrons at centre + sigma N(0,1)^3 (the initial electrons of the
 * paper's streamer runs, section "Simulation conditions"; draws outside the domain are
 * discarded).  NEUTRAL: per cell a Poisson number of electron-ion pairs of mean
 * n(x_c) dV, the electrons made by the coupling rule of eq. w (weights N div M,
 * remainder on the first, uniform in the cell) and as many positive ions.
 * Enqueued on the context's stream.  Errors: EINVAL (sigma <= 0, unknown kind); a full
 * bank drops the rest and is reported as ECAPACITY by itokmc_diagnostics. */
int itokmc_seed_particles(itokmc_ctx* ctx, const itokmc_seed_desc* seed);

/* Advance nsteps full steps of length dt (final algorithm, steps 1-8).  Returns
 * ENOCONV if a field solve missed its tolerance.  A particle-capacity overflow drops
 * the particles that do not fit, sets a device flag and is reported as ECAPACITY by
 * itokmc_diagnostics (the state stays consistent but incomplete). */
int itokmc_step(itokmc_ctx* ctx, uint32_t nsteps, double dt);
/* The same steps under a stop rule evaluated on the device: at most nsteps steps, the
 * run ending after the first step that began with at least stop_particles live
 * particles (0: no particle rule).  Prescribed-field mode: no host synchronisation
 * between steps; all nsteps steps are enqueued and, once the rule has ended the run,
 * the kernels of the remaining steps return at entry; one synchronisation at the end.
 * Self-consistent mode (whose field solve synchronises every refinement cycle anyway):
 * the steps run one at a time and the host reads the device's 4-byte decision after
 * each, so no reduction of the state is needed.  Writes the number of steps taken to
 * *steps_done (the context's step counter and bank follow it).  EINVAL without
 * coefficients or for dt <= 0; errors of itokmc_step. */
int itokmc_step_until(itokmc_ctx* ctx, uint32_t nsteps, double dt, uint64_t stop_particles,
                      uint32_t* steps_done);

/* The two halves of one step: transport (steps 1-5 and removal at the faces) and
 * react (steps 6-8, then the step counter advances).  step == transport + react. */
int itokmc_transport(itokmc_ctx* ctx, double dt);
int itokmc_react(itokmc_ctx* ctx, double dt);

/* Dynamic time step.  The paper runs fixed steps and names CFL- or physics-based
 * stepping as its next step (section "Final algorithm", closing paragraph).  The rule
 * here takes the smallest of
 *   dt_max,
 *   c_drift dx / v(Emax)          drift CFL: no electron drifts more than c_drift cells,
 *   c_diff dx^2 / (2 D)           diffusive spread of sqrt(c_diff) cells per axis,
 *   c_ion / (alpha(Emax) v(Emax)) at most c_ion expected ionizations per electron,
 * with v(E) = mu(E) E and Emax the largest |E| over the cell centres of the field the
 * next step starts from (E^k; |E_uniform| in the prescribed-field mode).  A limit whose
 * factor is 0, or whose rate is zero, is off.  Emax bounds every particle's field (a
 * CIC interpolation is a convex combination of cell-centre values), so the drift and
 * ionization limits hold for every particle when v and alpha v grow with E, which
 * needs mu_b >= -1.  In the self-consistent mode the advection uses E^{k+1}, known only
 * after the step's solve, so there the drift limit is the CFL number of E^k. */
typedef struct {
  double dt_max;          /* upper bound (s), > 0                                   */
  double c_drift;         /* drift limit factor (cells), 0 = off                    */
  double c_diff;          /* diffusion limit factor (cells^2), 0 = off              */
  double c_ion;           /* ionization limit factor (per electron), 0 = off        */
} itokmc_dt_rule;

/* out[0] = dt of the next step, out[1] = Emax (V/m) (host array of 2).  In the
 * self-consistent mode before the first step, computes the initial field first: the
 * solve the first transport would make, which it then skips, so the step is the same
 * as without the query.  Synchronises the stream.  Errors: EINVAL (no coefficients,
 * dt_max <= 0, a negative or non-finite factor, mu_b < -1 with the drift or
 * ionization limit on), ENOCONV (initial solve), EHIP. */
int itokmc_stable_dt(itokmc_ctx* ctx, const itokmc_dt_rule* rule, double* out);

/* nsteps steps, each of the dt that itokmc_stable_dt gives at its start; dts (host
 * array of nsteps, may be NULL) receives them.  One synchronisation per step (the
 * query).  Errors as itokmc_stable_dt and itokmc_step. */
int itokmc_step_adaptive(itokmc_ctx* ctx, const itokmc_dt_rule* rule, uint32_t nsteps,
                         double* dts);

/* Write a per-cell quantity (selector ITOKMC_Q_*) to the device buffer dev_out of
 * ncell (x3 for FIRES) elements of the stated type, enqueued on the context's stream.
 * NGP weights (the reaction network's electron count of section "KMC-particle
 * coupling"), the CIC density and RHO (section "Charge deposition & interpolation",
 * cell-centred tent weights, clouds folded into the wall cells) are computed from the
 * current particles; PHI and E are the last field solve's (eq. poisson_simp).
 * dev_out is owned by the caller.  Errors: EINVAL (unknown selector; PHI/E in UNIFORM
 * mode), EHIP. */
int itokmc_deposit(itokmc_ctx* ctx, int what, void* dev_out);

/* Reductions and tallies (the integer charge sum(n+ - n_e - n-) in units of e is
 * conserved by every reaction of the paper's air table, so it changes only by
 * outflow); synchronises the stream.  Returns ECAPACITY when an overflow flag
 * (ITOKMC_OVF_*) is set, after filling host_out; EHIP for an earlier asynchronous
 * failure. */
int itokmc_diagnostics(itokmc_ctx* ctx, itokmc_diag* host_out);

/* Particle state exchange with host memory (checkpoint, parity resynchronisation):
 * the computational particles of section "Ito diffusion", each a cell, an offset in
 * [0,1)^3 inside it, an integer weight (physical electrons) and a 64-bit id.
 * get: *n receives the count of live particles; arrays (each may be NULL) must hold n
 * entries (offsets: 3 n doubles, x y z interleaved).  Call with all arrays NULL to
 * query n.  set: replaces all particles (a host copy, synchronous); w must be >= 1,
 * offsets in [0,1), cells valid (EINVAL otherwise, state unchanged); ECAPACITY if n
 * exceeds max_particles.  Both synchronise the stream. */
int itokmc_get_particles(itokmc_ctx* ctx, uint64_t* n, uint32_t* cell, double* off,
                         uint32_t* w, uint64_t* id);
int itokmc_set_particles(itokmc_ctx* ctx, uint64_t n, const uint32_t* cell,
                         const double* off, const uint32_t* w, const uint64_t* id);
/* Per-cell counts (which = ITOKMC_Q_NPLUS, NMINUS or NGAMMA), host uint32 arrays of
 * ncell entries: the ion species of the air table (section "Numerical tests") as
 * immobile counts at the cell centres, and the photons awaiting transport in the next
 * step (final algorithm, step 6).  EINVAL for another selector.  Synchronous. */
int itokmc_get_counts(itokmc_ctx* ctx, int which, uint32_t* host);
int itokmc_set_counts(itokmc_ctx* ctx, int which, const uint32_t* host);
/* Step counter k (a component of every random stream's counter). */
int itokmc_set_step(itokmc_ctx* ctx, uint32_t step);
/* Potential of eq. poisson_simp (host doubles, ncell, V); set_field also recomputes
 * E = -grad phi at the cell centres.  POISSON mode only (EINVAL otherwise).
 * Synchronous. */
int itokmc_get_field(itokmc_ctx* ctx, double* phi);
int itokmc_set_field(itokmc_ctx* ctx, const double* phi);

/* Performance parameters (results do not depend on them beyond the solver
 * tolerance): multigrid pre/post red-black sweeps per level (default 2/2, each 0..8,
 * sum >= 1), bottom-level sweeps (0 = automatic), capture of the refinement cycle in
 * a HIP graph (default on), linear-in-time extrapolation of the potential as the
 * initial guess (default on), and the finest level's storage order (0 default: split
 * red-black, each x row holding its cells of one colour in its first half and of the
 * other colour in its second, so that a one-colour sweep moves whole lines; 1: natural
 * order; both give identical results; a grid that cannot be coarsened always uses
 * natural order).  set_tuning copies the struct; EINVAL if out of range. */
typedef struct {
  int32_t mg_pre, mg_post, bottom_sweeps, use_graph, extrapolate, fine_layout;
} itokmc_tuning;
int itokmc_set_tuning(itokmc_ctx* ctx, const itokmc_tuning* tuning);
int itokmc_get_tuning(itokmc_ctx* ctx, itokmc_tuning* tuning);

/* Per-phase timing with HIP events recorded around each kernel phase on the
 * context's stream (off by default).  Phases: 0 push, 1 photons, 2 bin scan,
 * 3 scatter, 4 KMC, 5 coupling kernel (one wavefront per cell), 6 charge-deposit
 * kernel, 7 field solve (with the field from the potential), 8 field push, 9 recount,
 * 10 larger merge tiers, 11 deposit clearing and right-hand side, 12 finest-level
 * smoother launches (one colour each, inside the solve; one count per launch), 13 light
 * coupling pass (one lane per cell), 14 per-cell pass of the time-step rule's field bound
 * (one count per query), 15 ion transport (its three passes).  phase_times synchronises, writes accumulated
 * milliseconds and launch counts for the first n phases, and clears them if reset is
 * nonzero. */
int itokmc_set_profiling(itokmc_ctx* ctx, int on);
int itokmc_phase_times(itokmc_ctx* ctx, double* ms, uint64_t* calls, int n, int reset);

void itokmc_destroy(itokmc_ctx* ctx);
const char* itokmc_last_error(const itokmc_ctx* ctx);

/* ---- batched ensemble of independent realizations --------------------------------
 * Many independent realizations of the method (each with its own grid, coefficients,
 * key and run length) share one device arena and advance together: one ensemble step
 * advances every active realization by one step of its own dt (final algorithm, steps
 * 1-8 in the uniform-field form: push, binning, KMC, coupling of eq. w) with one
 * sequence of pool-wide kernels, replayed as a HIP graph.  Every random stream is
 * keyed by the realization's own (seed, realization) and local cell or particle id,
 * so a realization's result is bit-identical whether it runs alone, in any mix, or as
 * a single context (itokmc_init_grid + itokmc_step) with the same descriptor.
 *
 * Pools: realizations take grid cells in 4096-cell blocks from a cell pool and reserve
 * a particle quota (their descriptor's max_particles) from a particle pool; admission
 * fails with EAGAIN while either pool or the slot table is full.  Supported
 * realizations: field_mode UNIFORM, n_ppc 0 (no merge), kgamma_ratio 0 (no photons),
 * Gaussian electron seeds, the ensemble's precision.
 * Conventions are those of the context API above (status codes, caller-owned arena,
 * stream given at creation, not thread-safe). */
typedef struct itokmc_ens itokmc_ens;
enum { ITOKMC_SLOT_FREE = 0, ITOKMC_SLOT_ACTIVE = 1, ITOKMC_SLOT_DONE = 2,
       ITOKMC_SLOT_CAPPED = 3 };

typedef struct {
  int32_t max_slots;       /* realizations resident at once, 1..4096                  */
  int32_t precision;       /* ITOKMC_FP32 | ITOKMC_FP64, shared by all realizations    */
  uint64_t max_cells;      /* cell pool (rounded up to 4096-cell blocks), <= 2^31      */
  uint64_t max_particles;  /* particle pool per bank, <= 2^31 - 1                      */
} itokmc_ens_desc;

/* Run length of one admitted realization.  It is done after nsteps steps, or after
 * the first step that began with at least stop_particles live particles (0: never). */
typedef struct {
  double dt;               /* step length (s)                                         */
  uint32_t nsteps;
  uint32_t pad0;
  uint64_t stop_particles;
  uint64_t tag;            /* caller's request id, echoed by poll                    */
} itokmc_run_desc;

typedef struct {
  int32_t slot;
  int32_t state;           /* ITOKMC_SLOT_DONE, or ITOKMC_SLOT_CAPPED if the
                              realization's particle quota overflowed (its state is
                              valid up to the dropped products; it stops there)       */
  uint64_t tag;
  uint32_t steps;          /* steps run                                               */
  uint32_t pad0;
} itokmc_slot_event;

typedef struct {
  int32_t slots_used, slots_free;
  uint64_t cells_free;     /* unassigned pool cells                                   */
  uint64_t particles_free; /* unreserved particle quota                               */
  uint64_t pool_particles; /* particle slots in use in the pool bank                  */
  uint64_t steps;          /* ensemble steps run                                      */
} itokmc_ens_info;

/* Launch shapes of the ensemble step (results do not depend on them): threads per
 * block of the particle kernels (64..1024, multiple of 64) and their blocks per
 * compute unit (1..64), threads per block of the KMC kernel, coupling wavefronts per
 * compute unit (1..256), HIP graph replay (default on), and fused_per_cu: 0 runs the
 * step as its sequence of kernels; k = 1, 2 or 4 runs it as one persistent fused
 * kernel (push, counting sort, scatter, KMC, coupling and end of step separated by
 * device-wide barriers with bounded waits) of k 256-thread workgroups per compute unit,
 * compiled for the register budget that keeps all of them resident at once (set_tuning
 * returns EINVAL if the device cannot).  A barrier gives up after 4 s (the environment
 * variable ITOKMC_FUSED_WAIT_US, read at ensemble creation, sets another limit in
 * microseconds); the step then ends early, ITOKMC_OVF_BARRIER is raised and the next
 * poll returns EHIP. */
typedef struct {
  int32_t push_block, push_blocks_per_cu, kmc_block, couple_per_cu, use_graph, fused_per_cu;
} itokmc_ens_tuning;

size_t itokmc_ensemble_arena_bytes(const itokmc_ens_desc* desc);
/* arena: device pointer, 256-byte aligned, >= itokmc_ensemble_arena_bytes(desc). */
int itokmc_ensemble_create(itokmc_ens** out, const itokmc_ens_desc* desc, void* arena,
                           size_t arena_bytes, void* stream);
/* Admit one realization: grid descriptor (its max_particles is the quota it
 * reserves), coefficients, seed and run length.  Seeds its particles (enqueued) and
 * returns its slot.  EAGAIN: no free slot, cells or quota; EINVAL: unsupported
 * descriptor. */
int itokmc_ensemble_admit(itokmc_ens* ens, const itokmc_grid_desc* desc,
                          const itokmc_coeffs* coeffs, const itokmc_seed_desc* seed,
                          const itokmc_run_desc* run, int32_t* slot);
/* Enqueue nsteps ensemble steps (does not synchronise). */
int itokmc_ensemble_step(itokmc_ens* ens, uint32_t nsteps);
/* Synchronise and report realizations that finished since the last poll (at most
 * max events; the rest are reported by later polls).  ECAPACITY if the pool bank
 * overflowed (not reachable while quotas hold). */
int itokmc_ensemble_poll(itokmc_ens* ens, itokmc_slot_event* events, int32_t max,
                         int32_t* n_events);
/* Results of a resident realization (synchronises): diagnostics as for a context,
 * its particles (cells local to its grid; same array conventions as
 * itokmc_get_particles) and per-cell counts (ITOKMC_Q_NGP_WEIGHT, NPLUS, NMINUS). */
int itokmc_ensemble_result(itokmc_ens* ens, int32_t slot, itokmc_diag* out);
/* Diagnostics of n resident realizations at once (one pass over the pool): out[i]
 * for slots[i]. */
int itokmc_ensemble_results(itokmc_ens* ens, const int32_t* slots, int32_t n,
                            itokmc_diag* out);
int itokmc_ensemble_get_particles(itokmc_ens* ens, int32_t slot, uint64_t* n, uint32_t* cell,
                                  double* off, uint32_t* w, uint64_t* id);
int itokmc_ensemble_get_counts(itokmc_ens* ens, int32_t slot, int which, uint32_t* host);
/* Free a slot with its cells and quota (its particles are dropped by the next step). */
int itokmc_ensemble_release(itokmc_ens* ens, int32_t slot);
int itokmc_ensemble_info(itokmc_ens* ens, itokmc_ens_info* out);
int itokmc_ensemble_set_tuning(itokmc_ens* ens, const itokmc_ens_tuning* tuning);
int itokmc_ensemble_get_tuning(itokmc_ens* ens, itokmc_ens_tuning* tuning);
/* Pick the launch shapes by timing candidate shapes on the live ensemble: each trial
 * is a real ensemble step (results are unchanged), candidates are interleaved over
 * rounds; the fastest is kept.  Coordinates in turn: the particle kernels' block and
 * blocks per compute unit, the KMC block, the coupling grid, then the form of the step
 * (the kernel sequence, or the fused kernel at each budget the device keeps resident).
 * best_ms: the kept shape's mean step time. */
int itokmc_ensemble_autotune(itokmc_ens* ens, uint32_t rounds, itokmc_ens_tuning* best,
                             double* best_ms);
void itokmc_ensemble_destroy(itokmc_ens* ens);
const char* itokmc_ensemble_last_error(const itokmc_ens* ens);

/* ---- kernel-level entry points (device pointers; used for unit parity) ----------
 * Philox4x32-10 (Salmon et al. 2011) blocks for counters (c0 + i, c1, c2, c3),
 * i < n, key (k0, k1): out is 4 n uint32. */
int itokmc_philox_fill(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                       uint32_t k1, uint64_t n, uint32_t* dev_out, void* stream);
/* One KMC step on n independent cells with the context's method parameters (section
 * "Reaction algorithm outline"): X (n x 4 int64: e, M+, M-, gamma; in/out), k (n x 5
 * double rates, 1/s: k_alpha, k_eta, k_gamma, k_ep, k_np), cell ids (n uint32, stream
 * keys), fires (n x 5 int64 out); all device pointers. */
int itokmc_kmc_cells(itokmc_ctx* ctx, uint64_t n, const uint32_t* dev_cell_ids,
                     int64_t* dev_X, const double* dev_k, double dt, uint32_t step,
                     int64_t* dev_fires);
/* Zero-dimensional reactors (section "Comparing reaction algorithms": a single cell's
 * reactions with no transport): nsteps consecutive KMC steps of length dt on each of n
 * independent reactors, in one launch.  Reactor i takes the steps step0 .. step0 +
 * nsteps - 1 of the stream (dev_cell_ids[i], step, KMC) under the key (context seed,
 * dev_realization[i]) (dev_realization may be NULL: the context's realization for all),
 * so its result does not depend on the other reactors of the call.  dev_nsteps (may be
 * NULL: nsteps for all) gives reactor i its own step count (steps past the 32-bit step
 * counter are not taken).  X (n x 4 int64: e, M+, M-, photons; in/out), k (n x 5 rates,
 * as itokmc_kmc_cells), fires (n x 5 int64 out: totals over the reactor's steps); all
 * device pointers.  Enqueued on the context's stream.  EINVAL on null arrays with
 * n > 0, dt <= 0, or step0 + nsteps beyond 2^32. */
int itokmc_kmc_run(itokmc_ctx* ctx, uint64_t n, const uint32_t* dev_cell_ids,
                   const uint32_t* dev_realization, const uint32_t* dev_nsteps, int64_t* dev_X,
                   const double* dev_k, double dt, uint32_t step0, uint32_t nsteps,
                   int64_t* dev_fires);

/* Counting sort of n particles by cell (the binning of particles into per-cell lists
 * that the reactions and superparticle management of the final algorithm, steps 7-8,
 * work on).  Inputs (device, n entries each): cell (u32), offsets ox, oy, oz (float for
 * ITOKMC_FP32, double for ITOKMC_FP64), weight w (u32; w == 0 marks a dead slot), id
 * (u64).  Outputs (device, capacity n each): the live particles (w > 0 and cell < ncell;
 * others are dropped) grouped by ascending cell, cell c occupying
 * [start[c], start[c+1]) with start of ncell + 1 u32; within a cell the order is
 * unspecified.  *n_out (device u32) receives the number of live particles.  Inputs and
 * outputs must not overlap.  workspace: device memory of at least
 * itokmc_sort_workspace_bytes(n, ncell) bytes, owned by the caller, unused after the
 * call's kernels finish.  Everything is enqueued on stream (a hipStream_t); nothing
 * synchronises.  Errors: EINVAL (null pointer, precision, ncell outside [1, 2^24], n >
 * 2^31 - 1), ENOMEM (workspace too small), EHIP. */
size_t itokmc_sort_workspace_bytes(uint64_t n, uint32_t ncell);
int itokmc_sort_by_cell(int precision, uint64_t n, uint32_t ncell, const uint32_t* cell,
                        const void* ox, const void* oy, const void* oz, const uint32_t* w,
                        const uint64_t* id, uint32_t* cell_out, void* ox_out, void* oy_out,
                        void* oz_out, uint32_t* w_out, uint64_t* id_out, uint32_t* start,
                        uint32_t* n_out, void* workspace, size_t workspace_bytes, void* stream);
/* The same sort without a workspace, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the scratch is a file-scope device array of 32 MiB per GPU, so the call
 * performs no allocation of any kind.  It accepts sizes whose
 * itokmc_sort_workspace_bytes(n, ncell) is at most 32 MiB (for example 2^20 cells with
 * 7e6 particles) and returns ECAPACITY beyond that.  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (on several streams or host threads) race
 * and must be serialised by the caller.  The first call on a device resolves the
 * array's address there (EHIP if that fails).  Other arguments and errors as
 * itokmc_sort_by_cell. */
int itokmc_sort_by_cell_noalloc(int precision, uint64_t n, uint32_t ncell,
                                const uint32_t* cell, const void* ox, const void* oy,
                                const void* oz, const uint32_t* w, const uint64_t* id,
                                uint32_t* cell_out, void* ox_out, void* oy_out, void* oz_out,
                                uint32_t* w_out, uint64_t* id_out, uint32_t* start,
                                uint32_t* n_out, void* stream);

#ifdef __cplusplus
}
#endif
#endif
