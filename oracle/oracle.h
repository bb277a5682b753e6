/*
 * Reference oracle for the Ito-KMC particle-mesh step (Marskar, "Stochastic and
 * self-consistent 3D modeling of streamer discharge trees with Kinetic Monte Carlo").
 *
 * TEST INFRASTRUCTURE ONLY.  This is a plain, slow, single-threaded FP64 C
 * implementation written from the paper, used to check the GPU library.  Only the
 * test suite, the smoke check and the CPU-baseline leg of the benchmark may load it.
 * It shares no code with the GPU library; the two are independent implementations
 * of the same definitions.
 *
 * Units: positions are stored in grid units (xi = X / dx, dimensionless), so that a
 * cell-relative offset o in [0,1) and cell index i give xi = i + o exactly.  Fields
 * are in V/m, times in s, weights are integer physical-particle counts.
 *
 * Parity status per function is listed in the header of each source file.
 */
#ifndef ITOKMC_ORACLE_H
#define ITOKMC_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Philox4x32-10 counter tags (top byte of counter word 3). */
enum {
  OR_TAG_PUSH = 1, OR_TAG_SEED = 2, OR_TAG_KMC = 3, OR_TAG_CREATE = 4,
  OR_TAG_PHOTON = 5, OR_TAG_ION = 6, OR_TAG_CONFIG = 7, OR_TAG_ARRIVAL = 8
};

/* Particle id kinds (bits 63:62). */
enum { OR_KIND_SEED = 0, OR_KIND_KMC = 1, OR_KIND_PHOTO = 2, OR_KIND_MERGE = 3 };

enum { OR_FIELD_UNIFORM = 0, OR_FIELD_POISSON = 1 };
enum { OR_KMC_HYBRID = 0, OR_KMC_PURE_TAU = 1 };
/* Particle shape for the field coupling (deposit and interpolation alike). */
enum { OR_SHAPE_CIC = 0, OR_SHAPE_TSC = 1 };

typedef struct {
  int32_t nx, ny, nz;      /* cells per axis                                   */
  int32_t field_mode;      /* OR_FIELD_UNIFORM | OR_FIELD_POISSON              */
  double dx;               /* cell edge, m                                     */
  double E_uniform[3];     /* prescribed field, V/m (uniform mode)             */
  double V_anode;          /* potential at z = L, V (Poisson mode); 0 at z = 0 */
  int32_t kmc_mode;        /* OR_KMC_HYBRID | OR_KMC_PURE_TAU                  */
  int32_t n_ppc;           /* target particles per cell; 0 disables merge/split */
  int32_t n_new;           /* max new computational particles per cell (64)    */
  int32_t kmc_nc;          /* critical threshold N_c (5)                       */
  int32_t kmc_nssa;        /* max SSA steps in the SSA exception (10)          */
  int32_t shape;           /* OR_SHAPE_CIC | OR_SHAPE_TSC (Poisson mode)       */
  double kmc_eps;          /* accuracy factor; INFINITY = accept any leap      */
  uint32_t seed, realization; /* Philox key                                    */
  double poisson_rtol;     /* linear-solve relative residual target            */
} or_desc;

typedef struct {
  double mu_a, mu_E0, mu_b;   /* mu(E) = mu_a * (E / mu_E0)^mu_b, m^2/(V s)     */
  double E_floor;             /* |E| clamp used inside mu(E), V/m               */
  double D;                   /* diffusion coefficient, m^2/s                   */
  double alpha_A, alpha_B;    /* alpha(E) = alpha_A * exp(-alpha_B / E), 1/m    */
  double eta;                 /* attachment coefficient, 1/m                    */
  double kgamma_ratio;        /* k_gamma = kgamma_ratio * k_alpha               */
  double photon_l1, photon_l2;/* absorption length log-uniform in [l1, l2], m   */
  /* recombination (0 disables each reaction):
   *   k_ep = beta_ep * T_e^beta_ep_b / dV with T_e = max(300 K, Te_a (E/mu_E0)^Te_b) K,
   *   k_np = beta_np / dV (beta_np at the gas temperature, 300 K)                 */
  double beta_ep, beta_ep_b, Te_a, Te_b, beta_np;
  /* ion transport (0 and 0: immobile ions): ion mobility, m^2/(V s), and ion
   * diffusion coefficient, m^2/s; positive ions drift along E, negative against */
  double mu_ion, D_ion;
} or_coeffs;

typedef struct {
  uint64_t n_particles, weight;     /* computational count, sum of weights       */
  int64_t n_plus, n_minus;          /* total ion counts                          */
  int64_t charge;                   /* sum(n+ - n_e - n-) in units of e          */
  uint64_t outflow_weight;          /* electron weight lost through domain faces */
  uint64_t fires[5];                /* cumulative fires: ionization, attachment, photon
                                       emission, electron-ion and ion-ion recombination */
  uint64_t photons_emitted, photons_absorbed, photons_lost; /* physical photons */
  uint64_t created, removed_weight; /* coupling tallies                          */
  uint64_t merged_cells;            /* cells rebuilt by merge/split              */
  uint32_t step;
  int32_t solver_iters;             /* last linear solve                          */
  double solver_relres;             /* last linear solve                          */
  uint64_t ion_outflow_plus, ion_outflow_minus; /* ions lost through domain faces */
} or_diag;

typedef struct or_sim or_sim;

/* ---- random numbers ------------------------------------------------------ */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
void or_normals3(uint64_t id, uint32_t step, uint32_t seed, uint32_t realization,
                 double out[3]);
/* Poisson(lambda) draws using a sequential per-cell stream (cell, step, tag). */
int64_t or_poisson_draw(double lambda, uint32_t cell, uint32_t step, uint32_t seed,
                        uint32_t realization, uint32_t* n_used);

/* ---- coefficients -------------------------------------------------------- */
double or_mobility(const or_coeffs* c, double Emag);
/* k = (k_alpha, k_eta, k_gamma, k_ep, k_np) at field magnitude Emag in a cell of
 * volume dV */
void or_rates(const or_coeffs* c, double Emag, double dV, double k[5]);

/* ---- KMC on independent cells (0-D) --------------------------------------- */
/* X: n_cells x 4 (e, M+, M-, gamma) in/out; k: n_cells x 5 rates (1/s);
 * fires: n_cells x 5 out.  Cell c draws from stream (cell_ids[c], step). */
void or_kmc_cells(const or_desc* d, int64_t n_cells, const uint32_t* cell_ids,
                  int64_t* X, const double* k, double dt, uint32_t step, int64_t* fires);
/* Step 4's non-critical leap bound dtau_nc for state X (e, M+, M-, gamma), rates k[5]. */
double or_kmc_leap_bound(const or_desc* d, const int64_t X[4], const double k[5]);

/* ---- merge/split of one cell ----------------------------------------------
 * off: m x 3 cell-relative offsets in [0,1); w, id: m.  Output leaves written to
 * out_off (n_out x 3), out_w, out_id; returns the number of leaves.  The leaf ids
 * are (MERGE, step, cell, leaf). */
int32_t or_merge_cell(int32_t n_ppc, int32_t m, const double* off, const uint64_t* w,
                      const uint64_t* id, uint32_t cell, uint32_t step,
                      double* out_off, uint64_t* out_w, uint64_t* out_id);

/* ---- simulation ------------------------------------------------------------ */
or_sim* or_create(const or_desc* d, const or_coeffs* c, uint64_t capacity);
void or_destroy(or_sim* s);
int or_seed_gaussian(or_sim* s, uint64_t n0, const double centre[3], double sigma);
int or_seed_neutral(or_sim* s, double n_peak, const double centre[3], double sigma);
int or_set_particles(or_sim* s, uint64_t n, const double* xi, const uint64_t* w,
                     const uint64_t* id);
uint64_t or_num_particles(const or_sim* s);
void or_get_particles(const or_sim* s, double* xi, uint64_t* w, uint64_t* id);
/* which: 0 = n_plus, 1 = n_minus, 2 = n_gamma (pending photons); int64 per cell */
void or_set_counts(or_sim* s, int which, const int64_t* v);
void or_get_counts(const or_sim* s, int which, int64_t* v);
void or_set_step(or_sim* s, uint32_t step);
/* Phase split of one step, following the paper's final algorithm:
 *   transport = conductivity, diffusive advance, field solve, advection, removal;
 *   react     = photon transport, reactions, coupling, superparticle management. */
int or_transport(or_sim* s, double dt);
int or_react(or_sim* s, double dt);
int or_step(or_sim* s, double dt, uint32_t nsteps);
void or_diagnostics(const or_sim* s, or_diag* out);

/* ---- dynamic time step (see sim.c) ---------------------------------------------- */
typedef struct {
  double dt_max;   /* upper bound, s (> 0)                                           */
  double c_drift;  /* dt <= c_drift dx / v(Emax); off when <= 0                      */
  double c_diff;   /* dt <= c_diff dx^2 / (2 D); off when <= 0 or D == 0             */
  double c_ion;    /* dt <= c_ion / (alpha(Emax) v(Emax)); off when <= 0 or no rate   */
} or_dt_rule;
/* Largest |E| over the cell centres of the field the next step starts from (uniform
 * mode: |E_uniform|); in the Poisson mode the initial field is computed first when
 * there is none yet (the same solve the first transport would make). */
double or_field_max(or_sim* s);
/* The next step's dt under rule r; Emax (may be NULL) receives the field bound. */
double or_stable_dt(or_sim* s, const or_dt_rule* r, double* Emax);
/* nsteps steps, each with the dt of or_stable_dt; dts (may be NULL) receives them. */
int or_step_adaptive(or_sim* s, const or_dt_rule* r, uint32_t nsteps, double* dts);
/* per-cell electron weight (NGP) of the current particles, int64 per cell */
void or_ngp_weight(const or_sim* s, int64_t* out);
/* electron number density (m^-3) of the current particles with the descriptor's shape
 * (CIC unless d->shape is TSC) */
void or_cic_density(const or_sim* s, double* out);
/* space charge (C/m^3) of the current state: e (n+ - n-) / dV - e n_e(CIC) */
void or_charge_density(const or_sim* s, double* out);
/* last per-cell fire counts (3 per cell) of the most recent react phase */
void or_get_fires(const or_sim* s, int64_t* out);

/* ---- field ----------------------------------------------------------------- */
/* Solve div(eps_r grad phi) = -rho / eps0 with phi(z=0) = 0, phi(z=L) = V_anode,
 * homogeneous Neumann on x and y faces, for cell-centred rho (C/m^3) and eps_r.
 * phi is the initial guess on entry.  Returns iterations; *relres out. */
int or_solve_poisson(const or_desc* d, const double* rho, const double* eps_r,
                     double* phi, double rtol, int max_iter, double* relres);
/* Cell-centred E = -grad phi using the boundary conditions above. */
void or_efield(const or_desc* d, const double* phi, double* Ex, double* Ey, double* Ez);
/* Access to the current field of a simulation (Poisson mode). */
void or_get_field(const or_sim* s, double* phi, double* Ex, double* Ey, double* Ez);
void or_set_field(or_sim* s, const double* phi);
/* Set the cell-centred field used by the next transport (as E^k) and reactions. */
void or_set_efield(or_sim* s, const double* Ex, const double* Ey, const double* Ez);
/* ||b - A phi|| / ||b|| of the system or_solve_poisson solves. */
double or_poisson_relres(const or_desc* d, const double* rho, const double* eps_r,
                         const double* phi);
/* Relative residual of phi in the semi-implicit system (eqs. conductivity and
 * poisson_simp) built from the simulation's particles X^k, ion counts, field E^k and
 * step k, as or_transport builds it; the state is unchanged. */
double or_semi_implicit_residual(const or_sim* s, double dt, const double* phi);
/* Semi-implicit update of n particles with given cell-centred E^k and E^{k+1}. */
void or_push_with_fields(const or_desc* d, const or_coeffs* c, uint64_t n, const double* xi,
                         const uint64_t* id, uint32_t step, double dt, const double* Ekx,
                         const double* Eky, const double* Ekz, const double* E1x,
                         const double* E1y, const double* E1z, double* out);

/* CIC helpers on an arbitrary point set (grid units). */
void or_cic_deposit(const or_desc* d, uint64_t n, const double* xi, const double* q,
                    double* grid);
void or_cic_interp(const or_desc* d, const double* grid, uint64_t n, const double* xi,
                   double* out);
/* TSC (quadratic B-spline) helpers, same conventions (see field.c). */
void or_tsc_deposit(const or_desc* d, uint64_t n, const double* xi, const double* q,
                    double* grid);
void or_tsc_interp(const or_desc* d, const double* grid, uint64_t n, const double* xi,
                   double* out);
/* The descriptor's shape (d->shape): CIC or TSC. */
void or_cloud_deposit(const or_desc* d, uint64_t n, const double* xi, const double* q,
                      double* grid);
void or_cloud_interp(const or_desc* d, const double* grid, uint64_t n, const double* xi,
                     double* out);

/* photon transport of one cell's pending photons; returns absorbed count and fills
 * positions (grid units) and weights of the photo-electrons. */
/* raw sample of one computational photon: emission point (grid units), direction,
 * absorption distance (m) */
void or_photon_sample(const or_desc* d, const or_coeffs* c, uint32_t cell, uint32_t slot,
                      uint32_t step, double y0[3], double dir[3], double* r_m);
int32_t or_photons_cell(const or_desc* d, const or_coeffs* c, uint32_t cell, int64_t n_gamma,
                        uint32_t step, double* xi_out, uint64_t* w_out, uint64_t* id_out,
                        uint64_t* lost_weight);

#ifdef __cplusplus
}
#endif
#endif
