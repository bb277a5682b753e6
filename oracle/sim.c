/*
 * Oracle: one Ito-KMC time step on a uniform grid (test infrastructure; see oracle.h).
 *
 * Step order follows the paper's "Final algorithm" (eight steps, Godunov split):
 *   transport: 1 conductivity sigma^k, 2 diffusive advance X_dagger, 3 rho_dagger and
 *              the semi-implicit field solve, 4 velocities from E^{k+1}(X^k),
 *              5 advection; particles outside the domain are removed;
 *   react:     6 photon transport (eq. photon_transport), 7 reactions (KMC) and the
 *              KMC-particle coupling of eq. w, 8 superparticle management.
 * In the prescribed-field mode steps 1-5 collapse to the standard Euler-Maruyama
 * update X += dt V + sqrt(2 D dt) N with V = -mu(E) E for electrons (eq. Vk1 with
 * sgn(Z) = -1).
 *
 * Readings where the text is silent:
 *   - ions are per-cell counts located at cell centres (the paper moves them as
 *     particles; their mobility is not given): immobile unless an ion mobility or
 *     diffusion coefficient is set, when they move on the grid as a lattice jump
 *     process (move_ions);
 *   - particles that leave any domain face are removed and their weight tallied;
 *   - mobility inside eq. Vk1 is mu^k = mu(|E^k(X^k)|); D is constant;
 *   - photons counted by the reactions of step k are transported in step k+1
 *     (step 6 precedes step 7); each absorbed photon of weight w makes one electron
 *     of weight w at the absorption point and w positive ions in that cell;
 *   - KMC products: net change dN of the cell's electrons; dN > 0 makes
 *     min(dN, N_new) particles of weight dN div M uniformly in the cell, the
 *     remainder going to the first; dN < 0 removes weight from the cell's particles
 *     in ascending id order;
 *   - merge/split runs in a cell holding more than N_ppc particles, or fewer with some
 *     weight >= 2;
 *   - the initial field (Poisson mode) is the solution for the present charge with
 *     sigma = 0;
 *   - the mobility formula is evaluated at max(|E|, E_floor);
 *   - with the TSC shape (a higher-order deposit, future work in the paper) the ions,
 *     point charges at their cell centres, are deposited with the same shape as the
 *     electrons, so a plasma of both on the same centres stays neutral.
 * Counter-based random streams (Philox key = (seed, realization)):
 *   push normals (id, step, PUSH); KMC (cell, step, KMC) sequential; creation
 *   (cell, slot, step, CREATE); photons (cell, slot, step, PHOTON sub 0/1); seeds
 *   (index, SEED sub 0), neutral seeds (cell, SEED sub 1) and (cell, slot, SEED sub 2).
 */
#include "or_internal.h"
#include <stdio.h>

static inline int64_t IDXS(const or_desc* d, int i, int j, int k) {
  return (int64_t)i + (int64_t)d->nx * ((int64_t)j + (int64_t)d->ny * k);
}

/* cell-centre field of cell c: the step's solved field, or the prescribed one */
static void field_at(const or_sim* s, int64_t c, double E[3]) {
  if (s->d.field_mode == OR_FIELD_UNIFORM) {
    for (int a = 0; a < 3; ++a) E[a] = s->d.E_uniform[a];
  } else {
    E[0] = s->Ex[c];
    E[1] = s->Ey[c];
    E[2] = s->Ez[c];
  }
}

uint64_t or_make_id(int kind, uint32_t step, uint32_t cell, uint32_t slot) {
  return ((uint64_t)kind << 62) | ((uint64_t)(step & 0x3FFFFFu) << 40) |
         ((uint64_t)(cell & 0xFFFFFFu) << 16) | (uint64_t)(slot & 0xFFFFu);
}

int32_t or_split_count(int64_t N, int32_t n_new, int64_t* w_base, int64_t* w_rem) {
  if (N <= 0) { *w_base = 0; *w_rem = 0; return 0; }
  int32_t M = N < (int64_t)n_new ? (int32_t)N : n_new;
  *w_base = N / M;
  *w_rem = N % M;
  return M;
}

double or_mobility(const or_coeffs* c, double Emag) {
  double E = Emag > c->E_floor ? Emag : c->E_floor;
  return c->mu_a * pow(E / c->mu_E0, c->mu_b);
}

/* Rates of the air-chemistry table: k_alpha = alpha mu E, k_eta = eta mu E,
 * k_gamma = ratio k_alpha; the recombination rates of the section on the chemistry,
 * k_ep = beta_ep(T_e) / dV and k_np = beta_np / dV, with the synthetic electron
 * temperature T_e(E) = max(300 K, Te_a (max(E, E_floor) / mu_E0)^Te_b) standing in for
 * the tabulated one. */
void or_rates(const or_coeffs* c, double Emag, double dV, double k[5]) {
  double mu = or_mobility(c, Emag);
  double alpha = Emag > 0.0 ? c->alpha_A * exp(-c->alpha_B / Emag) : 0.0;
  double v = mu * Emag;
  k[0] = alpha * v;
  k[1] = c->eta * v;
  k[2] = c->kgamma_ratio * k[0];
  k[3] = 0.0;
  if (c->beta_ep > 0.0) {
    double E = Emag > c->E_floor ? Emag : c->E_floor;
    double Te = fmax(300.0, c->Te_a * pow(E / c->mu_E0, c->Te_b));
    k[3] = c->beta_ep * pow(Te, c->beta_ep_b) / dV;
  }
  k[4] = c->beta_np > 0.0 ? c->beta_np / dV : 0.0;
}

int64_t or_cell_of(const or_desc* d, const double xi[3]) {
  if (!(xi[0] >= 0.0 && xi[0] < d->nx && xi[1] >= 0.0 && xi[1] < d->ny && xi[2] >= 0.0 &&
        xi[2] < d->nz))
    return -1;
  int64_t i = (int64_t)floor(xi[0]), j = (int64_t)floor(xi[1]), k = (int64_t)floor(xi[2]);
  return i + (int64_t)d->nx * (j + (int64_t)d->ny * k);
}

int or_push_particle(or_sim* s, const double xi[3], uint64_t w, uint64_t id) {
  if (s->np >= s->cap) {
    uint64_t nc = s->cap ? s->cap * 2 : 1024;
    or_particle* q = (or_particle*)realloc(s->p, sizeof(or_particle) * nc);
    if (!q) return -1;
    s->p = q;
    s->cap = nc;
  }
  or_particle* p = &s->p[s->np++];
  p->xi[0] = xi[0]; p->xi[1] = xi[1]; p->xi[2] = xi[2];
  p->w = w;
  p->id = id;
  return 0;
}

or_sim* or_create(const or_desc* d, const or_coeffs* c, uint64_t capacity) {
  or_sim* s = (or_sim*)calloc(1, sizeof(or_sim));
  s->d = *d;
  s->c = *c;
  s->ncell = (int64_t)d->nx * d->ny * d->nz;
  s->cap = capacity ? capacity : 1024;
  s->p = (or_particle*)malloc(sizeof(or_particle) * s->cap);
  s->nplus = (int64_t*)calloc((size_t)s->ncell, sizeof(int64_t));
  s->nminus = (int64_t*)calloc((size_t)s->ncell, sizeof(int64_t));
  s->ngamma = (int64_t*)calloc((size_t)s->ncell, sizeof(int64_t));
  s->fires = (int64_t*)calloc((size_t)s->ncell * 3, sizeof(int64_t));
  if (d->field_mode == OR_FIELD_POISSON) {
    s->phi = (double*)calloc((size_t)s->ncell, sizeof(double));
    s->Ex = (double*)calloc((size_t)s->ncell, sizeof(double));
    s->Ey = (double*)calloc((size_t)s->ncell, sizeof(double));
    s->Ez = (double*)calloc((size_t)s->ncell, sizeof(double));
  }
  return s;
}

void or_destroy(or_sim* s) {
  if (!s) return;
  free(s->p); free(s->nplus); free(s->nminus); free(s->ngamma); free(s->fires);
  free(s->phi); free(s->Ex); free(s->Ey); free(s->Ez);
  free(s);
}

/* ---- seeding ----------------------------------------------------------------- */

int or_seed_gaussian(or_sim* s, uint64_t n0, const double centre[3], double sigma) {
  const double two_pi = 6.283185307179586476925286766559;
  for (uint64_t i = 0; i < n0; ++i) {
    uint32_t x[4];
    or_block((uint32_t)i, (uint32_t)(i >> 32), 0, OR_TAG_SEED, 0, s->d.seed, s->d.realization, x);
    double r0 = sqrt(-2.0 * log(or_u_oc(x[0])));
    double t0 = two_pi * or_u_co(x[1]);
    double r1 = sqrt(-2.0 * log(or_u_oc(x[2])));
    double t1 = two_pi * or_u_co(x[3]);
    double n[3] = {r0 * cos(t0), r0 * sin(t0), r1 * cos(t1)};
    double xi[3];
    for (int a = 0; a < 3; ++a) xi[a] = (centre[a] + sigma * n[a]) / s->d.dx;
    if (or_cell_of(&s->d, xi) < 0) continue; /* draws outside the domain are discarded */
    if (or_push_particle(s, xi, 1, (1ull << 61) | i)) return -1;
  }
  s->field_valid = 0;
  return 0;
}

int or_seed_neutral(or_sim* s, double n_peak, const double centre[3], double sigma) {
  const or_desc* d = &s->d;
  double dV = d->dx * d->dx * d->dx;
  for (int k = 0; k < d->nz; ++k)
    for (int j = 0; j < d->ny; ++j)
      for (int i = 0; i < d->nx; ++i) {
        uint32_t c = (uint32_t)(i + d->nx * (j + d->ny * k));
        double x = (i + 0.5) * d->dx - centre[0];
        double y = (j + 0.5) * d->dx - centre[1];
        double z = (k + 0.5) * d->dx - centre[2];
        double lam = n_peak * exp(-(x * x + y * y + z * z) / (2.0 * sigma * sigma)) * dV;
        or_stream st;
        or_stream_init(&st, c, 0, OR_TAG_SEED, 1, d->seed, d->realization);
        int64_t N = or_poisson(lam, &st);
        if (N <= 0) continue;
        int64_t wb, wr;
        int32_t M = or_split_count(N, d->n_new, &wb, &wr);
        for (int32_t sl = 0; sl < M; ++sl) {
          uint32_t u[4];
          or_block(c, (uint32_t)sl, 0, OR_TAG_SEED, 2, d->seed, d->realization, u);
          double xi[3] = {i + or_u24(u[0]), j + or_u24(u[1]), k + or_u24(u[2])};
          uint64_t w = (uint64_t)(wb + (sl == 0 ? wr : 0));
          if (or_push_particle(s, xi, w, ((uint64_t)c << 16) | (uint64_t)sl)) return -1;
        }
        s->nplus[c] += N;
      }
  s->field_valid = 0;
  return 0;
}

/* ---- state access -------------------------------------------------------------- */

int or_set_particles(or_sim* s, uint64_t n, const double* xi, const uint64_t* w,
                     const uint64_t* id) {
  s->np = 0;
  for (uint64_t i = 0; i < n; ++i)
    if (or_push_particle(s, xi + 3 * i, w[i], id[i])) return -1;
  return 0;
}

uint64_t or_num_particles(const or_sim* s) { return s->np; }

void or_get_particles(const or_sim* s, double* xi, uint64_t* w, uint64_t* id) {
  for (uint64_t i = 0; i < s->np; ++i) {
    if (xi) for (int a = 0; a < 3; ++a) xi[3 * i + a] = s->p[i].xi[a];
    if (w) w[i] = s->p[i].w;
    if (id) id[i] = s->p[i].id;
  }
}

static int64_t* counts_ptr(const or_sim* s, int which) {
  return which == 0 ? s->nplus : which == 1 ? s->nminus : s->ngamma;
}
void or_set_counts(or_sim* s, int which, const int64_t* v) {
  memcpy(counts_ptr(s, which), v, sizeof(int64_t) * (size_t)s->ncell);
}
void or_get_counts(const or_sim* s, int which, int64_t* v) {
  memcpy(v, counts_ptr(s, which), sizeof(int64_t) * (size_t)s->ncell);
}
void or_set_step(or_sim* s, uint32_t step) { s->step = step; }
void or_get_fires(const or_sim* s, int64_t* out) {
  memcpy(out, s->fires, sizeof(int64_t) * 3 * (size_t)s->ncell);
}

/* ---- deposits ------------------------------------------------------------------- */

void or_ngp_weight(const or_sim* s, int64_t* out) {
  memset(out, 0, sizeof(int64_t) * (size_t)s->ncell);
  for (uint64_t i = 0; i < s->np; ++i) {
    int64_t c = or_cell_of(&s->d, s->p[i].xi);
    if (c >= 0) out[c] += (int64_t)s->p[i].w;
  }
}

static double* xi_array(const or_sim* s) {
  double* xi = (double*)malloc(sizeof(double) * 3 * (s->np ? s->np : 1));
  for (uint64_t i = 0; i < s->np; ++i)
    for (int a = 0; a < 3; ++a) xi[3 * i + a] = s->p[i].xi[a];
  return xi;
}

void or_cic_density(const or_sim* s, double* out) {
  double dV = s->d.dx * s->d.dx * s->d.dx;
  memset(out, 0, sizeof(double) * (size_t)s->ncell);
  double* xi = xi_array(s);
  double* q = (double*)malloc(sizeof(double) * (s->np ? s->np : 1));
  for (uint64_t i = 0; i < s->np; ++i) q[i] = (double)s->p[i].w / dV;
  or_cloud_deposit(&s->d, s->np, xi, q, out);
  free(xi);
  free(q);
}

/* ---- field (Poisson mode) -------------------------------------------------------- */

/* rho at cell centres from electron positions xi and the ion counts.  The ions are
 * point charges at their cell centres, deposited with the particles' shape: with CIC
 * that is their own cell (NGP); with TSC they spread over the 27 nearest centres like
 * any particle sitting on a centre. */
static void charge_density(const or_sim* s, const double* xi, double* rho) {
  double dV = s->d.dx * s->d.dx * s->d.dx;
  double* ne = (double*)calloc((size_t)s->ncell, sizeof(double));
  double* q = (double*)malloc(sizeof(double) * (s->np ? s->np : 1));
  if (s->d.shape != OR_SHAPE_TSC) {
    for (uint64_t i = 0; i < s->np; ++i) q[i] = (double)s->p[i].w / dV;
    or_cic_deposit(&s->d, s->np, xi, q, ne);
    for (int64_t c = 0; c < s->ncell; ++c)
      rho[c] = OR_E_CHARGE * ((double)(s->nplus[c] - s->nminus[c]) / dV - ne[c]);
  } else {
    /* counts in physical particles (integer charges times dyadic weights: the ion
     * sums are exact), scaled by the cell volume at the end */
    for (uint64_t i = 0; i < s->np; ++i) q[i] = (double)s->p[i].w;
    or_tsc_deposit(&s->d, s->np, xi, q, ne);
    double* ion = (double*)calloc((size_t)s->ncell, sizeof(double));
    double* pts = (double*)malloc(sizeof(double) * 3 * (size_t)s->ncell);
    double* qi = (double*)malloc(sizeof(double) * (size_t)s->ncell);
    for (int64_t c = 0; c < s->ncell; ++c) {
      const int64_t i = c % s->d.nx, j = (c / s->d.nx) % s->d.ny, k = c / ((int64_t)s->d.nx * s->d.ny);
      pts[3 * c + 0] = (double)i + 0.5;
      pts[3 * c + 1] = (double)j + 0.5;
      pts[3 * c + 2] = (double)k + 0.5;
      qi[c] = (double)(s->nplus[c] - s->nminus[c]);
    }
    or_tsc_deposit(&s->d, (uint64_t)s->ncell, pts, qi, ion);
    for (int64_t c = 0; c < s->ncell; ++c) rho[c] = OR_E_CHARGE * (ion[c] - ne[c]) / dV;
    free(ion); free(pts); free(qi);
  }
  free(ne);
  free(q);
}

void or_charge_density(const or_sim* s, double* out) {
  double* xi = xi_array(s);
  charge_density(s, xi, out);
  free(xi);
}

static int solve_field(or_sim* s, const double* rho, const double* eps_r) {
  double rr = 0.0;
  int it = or_solve_poisson(&s->d, rho, eps_r, s->phi, s->d.poisson_rtol, 100000, &rr);
  s->diag.solver_iters = it;
  s->diag.solver_relres = rr;
  or_efield(&s->d, s->phi, s->Ex, s->Ey, s->Ez);
  s->field_valid = 1;
  return 0;
}

static void initial_field(or_sim* s) {
  double* xi = xi_array(s);
  double* rho = (double*)malloc(sizeof(double) * (size_t)s->ncell);
  double* eps = (double*)malloc(sizeof(double) * (size_t)s->ncell);
  charge_density(s, xi, rho);
  for (int64_t c = 0; c < s->ncell; ++c) eps[c] = 1.0;
  solve_field(s, rho, eps);
  free(xi); free(rho); free(eps);
}

void or_get_field(const or_sim* s, double* phi, double* Ex, double* Ey, double* Ez) {
  size_t nb = sizeof(double) * (size_t)s->ncell;
  if (s->d.field_mode != OR_FIELD_POISSON) return;
  if (phi) memcpy(phi, s->phi, nb);
  if (Ex) memcpy(Ex, s->Ex, nb);
  if (Ey) memcpy(Ey, s->Ey, nb);
  if (Ez) memcpy(Ez, s->Ez, nb);
}

void or_set_efield(or_sim* s, const double* Ex, const double* Ey, const double* Ez) {
  if (s->d.field_mode != OR_FIELD_POISSON) return;
  size_t nb = sizeof(double) * (size_t)s->ncell;
  memcpy(s->Ex, Ex, nb);
  memcpy(s->Ey, Ey, nb);
  memcpy(s->Ez, Ez, nb);
  s->field_valid = 1;
}

void or_set_field(or_sim* s, const double* phi) {
  if (s->d.field_mode != OR_FIELD_POISSON) return;
  memcpy(s->phi, phi, sizeof(double) * (size_t)s->ncell);
  or_efield(&s->d, s->phi, s->Ex, s->Ey, s->Ez);
  s->field_valid = 1;
}

/* ---- transport ------------------------------------------------------------------- */

/* ---- ion transport -----------------------------------------------------------------
 * The paper moves ions as Ito particles (eq. Vk1 with sgn(Z) = +1 for positive ions)
 * and, in its future-work section, proposes treating heavy species as a continuum.
 * Reading taken: the ions stay per-cell integer counts (the reaction network's
 * populations) and drift and diffuse on the grid as a lattice jump process, the
 * first-order upwind finite-volume form of the drift-diffusion equation realised with
 * integer jumps.  An ion of sign q in a cell crosses the face towards its neighbour
 * along axis a in direction d (-1 or +1) at the rate
 *     max(0, d q mu_ion E_face,a) / dx + D_ion / dx^2,
 * with E_face the mean of the two cell-centre fields (the cell's own on a domain face).
 * Over a step the rates are frozen: with n the count before the move, face f (order
 * -x, +x, -y, +y, -z, +z) has the mean lambda_f = n rate_f dt, and the faces' counts are
 * independent Poisson(lambda_f) (tau leaping of the jump process).  They are drawn per
 * species (M+ then M-) in one of two equivalent ways, chosen by the total mean
 * Lambda = sum lambda_f (summed in face order):
 *   Lambda < 10: the number of movers N ~ Poisson(Lambda), capped at n, from the stream
 *     (cell, step, ION, sub = species); each mover then picks its face with one more
 *     uniform u from that stream, the first face whose running sum of lambda exceeds
 *     u Lambda (a Poisson total split multinomially gives independent Poisson faces);
 *   otherwise: each face's Poisson(lambda_f) from its own stream (cell, step, ION,
 *     sub = 2 + 6 species + face), each capped at the ions not yet moved.
 * Most cells hold a few ions with a tiny Lambda: the first way costs them one block of
 * random words instead of six.  Ions crossing a domain face leave and are tallied.  The
 * field is the step's E^{k+1} (the uniform field in the prescribed mode): the ions move
 * explicitly, their dielectric relaxation time being far above dt. */
static void move_ions(or_sim* s, double dt) {
  const or_desc* d = &s->d;
  const or_coeffs* c = &s->c;
  if (!(c->mu_ion > 0.0) && !(c->D_ion > 0.0)) return;
  const int n3[3] = {d->nx, d->ny, d->nz};
  const double inv_dx = 1.0 / d->dx;
  const double dr = c->D_ion / (d->dx * d->dx);
  int64_t* nxt[2];
  nxt[0] = (int64_t*)calloc((size_t)s->ncell, sizeof(int64_t));
  nxt[1] = (int64_t*)calloc((size_t)s->ncell, sizeof(int64_t));
  const int64_t* cur[2] = {s->nplus, s->nminus};
  uint64_t out[2] = {0, 0};
  for (int k = 0; k < d->nz; ++k)
    for (int j = 0; j < d->ny; ++j)
      for (int i = 0; i < d->nx; ++i) {
        const int64_t c0 = IDXS(d, i, j, k);
        if (cur[0][c0] == 0 && cur[1][c0] == 0) continue;
        double Ec[3];
        field_at(s, c0, Ec);
        int64_t nb[6];
        double Ef[6];
        for (int f = 0; f < 6; ++f) {
          const int a = f / 2, dir = (f & 1) ? 1 : -1;
          int ijk[3] = {i, j, k};
          ijk[a] += dir;
          nb[f] = -1;
          Ef[f] = Ec[a];
          if (ijk[a] >= 0 && ijk[a] < n3[a]) {
            double En[3];
            nb[f] = IDXS(d, ijk[0], ijk[1], ijk[2]);
            field_at(s, nb[f], En);
            Ef[f] = 0.5 * (Ec[a] + En[a]);
          }
        }
        for (int sp = 0; sp < 2; ++sp) {
          const int64_t n0 = cur[sp][c0];
          if (n0 == 0) continue;
          const double q = sp == 0 ? 1.0 : -1.0;
          double lam[6], L = 0.0;
          for (int f = 0; f < 6; ++f) {
            const double dir = (f & 1) ? 1.0 : -1.0;
            const double v = q * c->mu_ion * Ef[f];
            const double rate = fmax(0.0, dir * v) * inv_dx + dr;
            lam[f] = (double)n0 * rate * dt;
            L += lam[f];
          }
          int64_t K[6] = {0, 0, 0, 0, 0, 0};
          if (!(L > 0.0)) {
            /* no movers */
          } else if (L < 10.0) {
            or_stream st;
            or_stream_init(&st, (uint32_t)c0, s->step, OR_TAG_ION, (uint32_t)sp, d->seed, d->realization);
            int64_t N = or_poisson(L, &st);
            if (N > n0) N = n0;
            for (int64_t m = 0; m < N; ++m) {
              const double t = or_u_co(or_stream_next(&st)) * L;
              int f = 0;
              double acc = lam[0];
              while (f < 5 && t >= acc) acc += lam[++f];
              K[f] += 1;
            }
          } else {
            int64_t left = n0;
            for (int f = 0; f < 6; ++f) {
              or_stream st;
              or_stream_init(&st, (uint32_t)c0, s->step, OR_TAG_ION, (uint32_t)(2 + 6 * sp + f), d->seed,
                             d->realization);
              int64_t kf = or_poisson(lam[f], &st);
              if (kf > left) kf = left;
              left -= kf;
              K[f] = kf;
            }
          }
          int64_t moved = 0;
          for (int f = 0; f < 6; ++f) {
            moved += K[f];
            if (nb[f] >= 0) nxt[sp][nb[f]] += K[f];
            else out[sp] += (uint64_t)K[f];
          }
          nxt[sp][c0] += n0 - moved;
        }
      }
  memcpy(s->nplus, nxt[0], sizeof(int64_t) * (size_t)s->ncell);
  memcpy(s->nminus, nxt[1], sizeof(int64_t) * (size_t)s->ncell);
  s->diag.ion_outflow_plus += out[0];
  s->diag.ion_outflow_minus += out[1];
  free(nxt[0]);
  free(nxt[1]);
}

static void remove_outside(or_sim* s) {
  uint64_t keep = 0;
  for (uint64_t i = 0; i < s->np; ++i) {
    if (or_cell_of(&s->d, s->p[i].xi) < 0) {
      s->diag.outflow_weight += s->p[i].w;
      continue;
    }
    s->p[keep++] = s->p[i];
  }
  s->np = keep;
}

int or_transport(or_sim* s, double dt) {
  const or_desc* d = &s->d;
  const or_coeffs* c = &s->c;
  double diff = sqrt(2.0 * c->D * dt) / d->dx; /* grid units per unit normal */
  if (d->field_mode == OR_FIELD_UNIFORM) {
    const double* E = d->E_uniform;
    double Em = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
    double mu = or_mobility(c, Em);
    for (uint64_t i = 0; i < s->np; ++i) {
      double n[3];
      or_normals3(s->p[i].id, s->step, d->seed, d->realization, n);
      for (int a = 0; a < 3; ++a) s->p[i].xi[a] += (-mu * E[a] * dt) / d->dx + diff * n[a];
    }
    move_ions(s, dt);
    remove_outside(s);
    return 0;
  }
  /* semi-implicit Euler-Maruyama (final algorithm, steps 1-5) */
  if (!s->field_valid) initial_field(s);
  uint64_t np = s->np;
  double dV = d->dx * d->dx * d->dx;
  double* xk = xi_array(s);
  double* ex = (double*)malloc(sizeof(double) * (np ? np : 1));
  double* ey = (double*)malloc(sizeof(double) * (np ? np : 1));
  double* ez = (double*)malloc(sizeof(double) * (np ? np : 1));
  double* mu = (double*)malloc(sizeof(double) * (np ? np : 1));
  /* step 1: sigma^k = e sum_p mu_p w_p W / dV with mu_p = mu(|E^k(X_p^k)|) */
  or_cloud_interp(d, s->Ex, np, xk, ex);
  or_cloud_interp(d, s->Ey, np, xk, ey);
  or_cloud_interp(d, s->Ez, np, xk, ez);
  double* q = (double*)malloc(sizeof(double) * (np ? np : 1));
  for (uint64_t i = 0; i < np; ++i) {
    mu[i] = or_mobility(c, sqrt(ex[i] * ex[i] + ey[i] * ey[i] + ez[i] * ez[i]));
    q[i] = OR_E_CHARGE * mu[i] * (double)s->p[i].w / dV;
  }
  double* sigma = (double*)calloc((size_t)s->ncell, sizeof(double));
  or_cloud_deposit(d, np, xk, q, sigma);
  /* step 2: X_dagger = X^k + sqrt(2 D dt) N */
  for (uint64_t i = 0; i < np; ++i) {
    double n[3];
    or_normals3(s->p[i].id, s->step, d->seed, d->realization, n);
    for (int a = 0; a < 3; ++a) s->p[i].xi[a] += diff * n[a];
  }
  /* step 3: rho_dagger and the semi-implicit field solve */
  double* xd = xi_array(s);
  double* rho = (double*)malloc(sizeof(double) * (size_t)s->ncell);
  double* eps = (double*)malloc(sizeof(double) * (size_t)s->ncell);
  charge_density(s, xd, rho);
  for (int64_t cc = 0; cc < s->ncell; ++cc) eps[cc] = 1.0 + sigma[cc] * dt / OR_EPS0;
  solve_field(s, rho, eps);
  /* steps 4-5: V^{k+1} = -mu^k E^{k+1}(X^k); X^{k+1} = X_dagger + V dt */
  or_cloud_interp(d, s->Ex, np, xk, ex);
  or_cloud_interp(d, s->Ey, np, xk, ey);
  or_cloud_interp(d, s->Ez, np, xk, ez);
  for (uint64_t i = 0; i < np; ++i) {
    s->p[i].xi[0] += -mu[i] * ex[i] * dt / d->dx;
    s->p[i].xi[1] += -mu[i] * ey[i] * dt / d->dx;
    s->p[i].xi[2] += -mu[i] * ez[i] * dt / d->dx;
  }
  free(xk); free(ex); free(ey); free(ez); free(mu); free(q); free(sigma);
  free(xd); free(rho); free(eps);
  move_ions(s, dt);
  remove_outside(s);
  return 0;
}

/* Relative residual of a potential phi in the semi-implicit system built from the
 * simulation's state (particles X^k, ion counts, field E^k as set by or_set_efield,
 * step counter k): steps 1-3 of or_transport (sigma^k of eq. conductivity at X^k, the
 * diffusive advance X_dagger, rho_dagger, eq. poisson_simp) without solving.  The state
 * is not changed. */
double or_semi_implicit_residual(const or_sim* s, double dt, const double* phi) {
  const or_desc* d = &s->d;
  const or_coeffs* c = &s->c;
  uint64_t np = s->np;
  double dV = d->dx * d->dx * d->dx;
  double diff = sqrt(2.0 * c->D * dt) / d->dx;
  double* xk = xi_array(s);
  double* ex = (double*)malloc(sizeof(double) * (np ? np : 1));
  double* ey = (double*)malloc(sizeof(double) * (np ? np : 1));
  double* ez = (double*)malloc(sizeof(double) * (np ? np : 1));
  double* q = (double*)malloc(sizeof(double) * (np ? np : 1));
  or_cloud_interp(d, s->Ex, np, xk, ex);
  or_cloud_interp(d, s->Ey, np, xk, ey);
  or_cloud_interp(d, s->Ez, np, xk, ez);
  for (uint64_t i = 0; i < np; ++i) {
    double mu = or_mobility(c, sqrt(ex[i] * ex[i] + ey[i] * ey[i] + ez[i] * ez[i]));
    q[i] = OR_E_CHARGE * mu * (double)s->p[i].w / dV;
  }
  double* sigma = (double*)calloc((size_t)s->ncell, sizeof(double));
  or_cloud_deposit(d, np, xk, q, sigma);
  double* xd = (double*)malloc(sizeof(double) * 3 * (np ? np : 1));
  for (uint64_t i = 0; i < np; ++i) {
    double n[3];
    or_normals3(s->p[i].id, s->step, d->seed, d->realization, n);
    for (int a = 0; a < 3; ++a) xd[3 * i + a] = xk[3 * i + a] + diff * n[a];
  }
  double* rho = (double*)malloc(sizeof(double) * (size_t)s->ncell);
  double* eps = (double*)malloc(sizeof(double) * (size_t)s->ncell);
  charge_density(s, xd, rho);
  for (int64_t cc = 0; cc < s->ncell; ++cc) eps[cc] = 1.0 + sigma[cc] * dt / OR_EPS0;
  double rr = or_poisson_relres(d, rho, eps, phi);
  free(xk); free(ex); free(ey); free(ez); free(q); free(sigma); free(xd); free(rho); free(eps);
  return rr;
}

/* The semi-implicit update of final-algorithm steps 2, 4 and 5 for n particles with
 * given cell-centred fields E^k and E^{k+1} (three arrays each):
 * X^{k+1} = X^k + sqrt(2 D dt) N(id, k) - mu(|E^k(X^k)|) E^{k+1}(X^k) dt (grid units). */
void or_push_with_fields(const or_desc* d, const or_coeffs* c, uint64_t n, const double* xi,
                         const uint64_t* id, uint32_t step, double dt, const double* Ekx,
                         const double* Eky, const double* Ekz, const double* E1x,
                         const double* E1y, const double* E1z, double* out) {
  double diff = sqrt(2.0 * c->D * dt) / d->dx;
  for (uint64_t i = 0; i < n; ++i) {
    const double* x = xi + 3 * i;
    double ek[3], e1[3], nrm[3];
    or_cloud_interp(d, Ekx, 1, x, &ek[0]);
    or_cloud_interp(d, Eky, 1, x, &ek[1]);
    or_cloud_interp(d, Ekz, 1, x, &ek[2]);
    or_cloud_interp(d, E1x, 1, x, &e1[0]);
    or_cloud_interp(d, E1y, 1, x, &e1[1]);
    or_cloud_interp(d, E1z, 1, x, &e1[2]);
    double mu = or_mobility(c, sqrt(ek[0] * ek[0] + ek[1] * ek[1] + ek[2] * ek[2]));
    or_normals3(id[i], step, d->seed, d->realization, nrm);
    for (int a = 0; a < 3; ++a) out[3 * i + a] = (x[a] + diff * nrm[a]) + (-mu * e1[a] * dt / d->dx);
  }
}

/* ---- photons (final algorithm step 6) ------------------------------------------ */

void or_photon_sample(const or_desc* d, const or_coeffs* c, uint32_t cell, uint32_t slot,
                      uint32_t step, double y0[3], double dir[3], double* r_m) {
  const double two_pi = 6.283185307179586476925286766559;
  int ci = (int)(cell % (uint32_t)d->nx);
  int cj = (int)((cell / (uint32_t)d->nx) % (uint32_t)d->ny);
  int ck = (int)(cell / ((uint32_t)d->nx * (uint32_t)d->ny));
  uint32_t A[4], B[4];
  or_block(cell, slot, step, OR_TAG_PHOTON, 0, d->seed, d->realization, A);
  or_block(cell, slot, step, OR_TAG_PHOTON, 1, d->seed, d->realization, B);
  y0[0] = ci + or_u24(A[0]);
  y0[1] = cj + or_u24(A[1]);
  y0[2] = ck + or_u24(A[2]);
  double cth = 2.0 * or_u_co(A[3]) - 1.0;            /* uniform on the sphere */
  double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
  double phi = two_pi * or_u_co(B[0]);
  dir[0] = sth * cos(phi);
  dir[1] = sth * sin(phi);
  dir[2] = cth;
  /* mean absorption length log-uniform in [l1, l2]; distance exponential */
  double ell = c->photon_l1 * pow(c->photon_l2 / c->photon_l1, or_u_co(B[1]));
  *r_m = -ell * log(or_u_oc(B[2]));
}

int32_t or_photons_cell(const or_desc* d, const or_coeffs* c, uint32_t cell, int64_t n_gamma,
                        uint32_t step, double* xi_out, uint64_t* w_out, uint64_t* id_out,
                        uint64_t* lost_weight) {
  int64_t wb, wr;
  int32_t M = or_split_count(n_gamma, d->n_new, &wb, &wr);
  int32_t n_abs = 0;
  for (int32_t sl = 0; sl < M; ++sl) {
    uint64_t w = (uint64_t)(wb + (sl == 0 ? wr : 0));
    double y0[3], dir[3], r;
    or_photon_sample(d, c, cell, (uint32_t)sl, step, y0, dir, &r);
    double rg = r / d->dx; /* grid units */
    double y[3] = {y0[0] + rg * dir[0], y0[1] + rg * dir[1], y0[2] + rg * dir[2]};
    if (or_cell_of(d, y) < 0) {   /* photons leaving the domain are removed */
      if (lost_weight) *lost_weight += w;
      continue;
    }
    for (int a = 0; a < 3; ++a) xi_out[3 * n_abs + a] = y[a];
    w_out[n_abs] = w;
    id_out[n_abs] = or_make_id(OR_KIND_PHOTO, step, cell, (uint32_t)sl);
    n_abs++;
  }
  return n_abs;
}

static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return x < y ? -1 : x > y ? 1 : 0;
}

typedef struct { uint64_t id; uint64_t idx; } idpair;
static int cmp_idpair(const void* a, const void* b) {
  return cmp_u64(&((const idpair*)a)->id, &((const idpair*)b)->id);
}

/* ---- react: photons, KMC, coupling, superparticles ------------------------------ */

int or_react(or_sim* s, double dt) {
  const or_desc* d = &s->d;
  const or_coeffs* c = &s->c;
  uint32_t step = s->step;
  int64_t ncell = s->ncell;
  double* xbuf = (double*)malloc(sizeof(double) * 3 * 64 * (size_t)(d->n_new > 64 ? d->n_new : 64));
  uint64_t* wbuf = (uint64_t*)malloc(sizeof(uint64_t) * 64 * (size_t)(d->n_new > 64 ? d->n_new : 64));
  uint64_t* ibuf = (uint64_t*)malloc(sizeof(uint64_t) * 64 * (size_t)(d->n_new > 64 ? d->n_new : 64));

  /* step 6: photons emitted during the previous step */
  for (int64_t cc = 0; cc < ncell; ++cc) {
    int64_t ng = s->ngamma[cc];
    if (ng <= 0) continue;
    uint64_t lost = 0;
    int32_t na = or_photons_cell(d, c, (uint32_t)cc, ng, step, xbuf, wbuf, ibuf, &lost);
    for (int32_t i = 0; i < na; ++i) {
      or_push_particle(s, xbuf + 3 * i, wbuf[i], ibuf[i]);
      s->nplus[or_cell_of(d, xbuf + 3 * i)] += (int64_t)wbuf[i];
      s->diag.photons_absorbed += wbuf[i];
    }
    s->diag.photons_lost += lost;
    s->ngamma[cc] = 0;
  }

  /* per-cell particle lists (CSR by cell) */
  int64_t* start = (int64_t*)calloc((size_t)ncell + 1, sizeof(int64_t));
  for (uint64_t i = 0; i < s->np; ++i) start[or_cell_of(d, s->p[i].xi) + 1] += 1;
  for (int64_t cc = 0; cc < ncell; ++cc) start[cc + 1] += start[cc];
  idpair* order = (idpair*)malloc(sizeof(idpair) * (s->np ? s->np : 1));
  int64_t* fill = (int64_t*)calloc((size_t)ncell, sizeof(int64_t));
  for (uint64_t i = 0; i < s->np; ++i) {
    int64_t cc = or_cell_of(d, s->p[i].xi);
    int64_t pos = start[cc] + fill[cc]++;
    order[pos].id = s->p[i].id;
    order[pos].idx = i;
  }
  free(fill);

  /* rates: prescribed field, or |E^{k+1}| at the cell centre */
  const double dV = d->dx * d->dx * d->dx;
  double kuni[5];
  if (d->field_mode == OR_FIELD_UNIFORM) {
    const double* E = d->E_uniform;
    or_rates(c, sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]), dV, kuni);
  }
  memset(s->fires, 0, sizeof(int64_t) * 3 * (size_t)ncell);
  uint64_t np_before = s->np;
  char* dead = (char*)calloc(np_before ? np_before : 1, 1);
  uint64_t n_new_total = 0;
  or_particle* created = NULL;
  uint64_t created_cap = 0;

  for (int64_t cc = 0; cc < ncell; ++cc) {
    int64_t b = start[cc], e = start[cc + 1];
    /* step 7 acts on every cell where a reaction can fire: one holding electrons, or
     * (ion-ion recombination) one holding ions of both signs */
    if (e == b && !(c->beta_np > 0.0 && s->nplus[cc] > 0 && s->nminus[cc] > 0)) continue;
    /* step 7: reactions on the NGP state of the cell */
    int64_t Xe = 0;
    for (int64_t q = b; q < e; ++q) Xe += (int64_t)s->p[order[q].idx].w;
    int64_t X[4] = {Xe, s->nplus[cc], s->nminus[cc], 0};
    double k[5];
    if (d->field_mode == OR_FIELD_UNIFORM) memcpy(k, kuni, sizeof(k));
    else {
      double Ex = s->Ex[cc], Ey = s->Ey[cc], Ez = s->Ez[cc];
      or_rates(c, sqrt(Ex * Ex + Ey * Ey + Ez * Ez), dV, k);
    }
    or_stream st;
    or_stream_init(&st, (uint32_t)cc, step, OR_TAG_KMC, 0, d->seed, d->realization);
    int64_t f[5];
    or_kmc_advance(d, X, k, dt, &st, f);
    for (int r = 0; r < 3; ++r) s->fires[3 * cc + r] = f[r];
    for (int r = 0; r < 5; ++r) s->diag.fires[r] += (uint64_t)f[r];
    s->nplus[cc] = X[1];
    s->nminus[cc] = X[2];
    s->ngamma[cc] = X[3];
    s->diag.photons_emitted += (uint64_t)X[3];
    int64_t dN = X[0] - Xe;

    /* coupling, eq. w */
    int32_t ncreated = 0;
    if (dN < 0) {
      qsort(order + b, (size_t)(e - b), sizeof(idpair), cmp_idpair);
      int64_t R = -dN;
      for (int64_t q = b; q < e && R > 0; ++q) {
        or_particle* p = &s->p[order[q].idx];
        int64_t take = (int64_t)p->w < R ? (int64_t)p->w : R;
        p->w -= (uint64_t)take;
        R -= take;
        s->diag.removed_weight += (uint64_t)take;
        if (p->w == 0) dead[order[q].idx] = 1;
      }
    } else if (dN > 0) {
      int64_t wb, wr;
      int32_t M = or_split_count(dN, d->n_new, &wb, &wr);
      int ci = (int)(cc % d->nx), cj = (int)((cc / d->nx) % d->ny), ck = (int)(cc / ((int64_t)d->nx * d->ny));
      if (n_new_total + (uint64_t)M > created_cap) {
        created_cap = (created_cap + (uint64_t)M) * 2;
        created = (or_particle*)realloc(created, sizeof(or_particle) * created_cap);
      }
      for (int32_t sl = 0; sl < M; ++sl) {
        uint32_t u[4];
        or_block((uint32_t)cc, (uint32_t)sl, step, OR_TAG_CREATE, 0, d->seed, d->realization, u);
        or_particle* p = &created[n_new_total + (uint64_t)sl];
        p->xi[0] = ci + or_u24(u[0]);
        p->xi[1] = cj + or_u24(u[1]);
        p->xi[2] = ck + or_u24(u[2]);
        p->w = (uint64_t)(wb + (sl == 0 ? wr : 0));
        p->id = or_make_id(OR_KIND_KMC, step, (uint32_t)cc, (uint32_t)sl);
      }
      ncreated = M;
      n_new_total += (uint64_t)M;
      s->diag.created += (uint64_t)M;
    }

    /* step 8: superparticle management */
    if (d->n_ppc > 0) {
      int64_t m_alive = 0;
      uint64_t wmax = 0;
      for (int64_t q = b; q < e; ++q) {
        if (dead[order[q].idx]) continue;
        m_alive++;
        if (s->p[order[q].idx].w > wmax) wmax = s->p[order[q].idx].w;
      }
      for (int32_t t = 0; t < ncreated; ++t) {
        m_alive++;
        if (created[n_new_total - (uint64_t)ncreated + (uint64_t)t].w > wmax)
          wmax = created[n_new_total - (uint64_t)ncreated + (uint64_t)t].w;
      }
      int trigger = m_alive > d->n_ppc || (m_alive < d->n_ppc && wmax >= 2);
      if (trigger && m_alive > 0) {
        double* off = (double*)malloc(sizeof(double) * 3 * (size_t)m_alive);
        uint64_t* ww = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m_alive);
        uint64_t* ii = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)m_alive);
        int64_t m = 0;
        int cidx[3] = {(int)(cc % d->nx), (int)((cc / d->nx) % d->ny), (int)(cc / ((int64_t)d->nx * d->ny))};
        for (int64_t q = b; q < e; ++q) {
          if (dead[order[q].idx]) continue;
          or_particle* p = &s->p[order[q].idx];
          for (int a = 0; a < 3; ++a) off[3 * m + a] = p->xi[a] - cidx[a];
          ww[m] = p->w; ii[m] = p->id; m++;
          dead[order[q].idx] = 1;
        }
        for (int32_t t = 0; t < ncreated; ++t) {
          or_particle* p = &created[n_new_total - (uint64_t)ncreated + (uint64_t)t];
          for (int a = 0; a < 3; ++a) off[3 * m + a] = p->xi[a] - cidx[a];
          ww[m] = p->w; ii[m] = p->id; m++;
        }
        n_new_total -= (uint64_t)ncreated; /* the created particles are consumed */
        int32_t cap = d->n_ppc;
        double* lo = (double*)malloc(sizeof(double) * 3 * (size_t)cap);
        uint64_t* lw = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
        uint64_t* li = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
        int32_t nl = or_merge_cell(d->n_ppc, (int32_t)m, off, ww, ii, (uint32_t)cc, step, lo, lw, li);
        if (n_new_total + (uint64_t)nl > created_cap) {
          created_cap = (created_cap + (uint64_t)nl) * 2;
          created = (or_particle*)realloc(created, sizeof(or_particle) * created_cap);
        }
        for (int32_t t = 0; t < nl; ++t) {
          or_particle* p = &created[n_new_total++];
          for (int a = 0; a < 3; ++a) p->xi[a] = cidx[a] + lo[3 * t + a];
          p->w = lw[t];
          p->id = li[t];
        }
        s->diag.merged_cells += 1;
        free(off); free(ww); free(ii); free(lo); free(lw); free(li);
      }
    }
  }
  /* compact survivors and append the new particles */
  uint64_t keep = 0;
  for (uint64_t i = 0; i < np_before; ++i)
    if (!dead[i]) s->p[keep++] = s->p[i];
  s->np = keep;
  for (uint64_t t = 0; t < n_new_total; ++t)
    or_push_particle(s, created[t].xi, created[t].w, created[t].id);
  free(created); free(dead); free(order); free(start);
  free(xbuf); free(wbuf); free(ibuf);
  s->step += 1;
  s->diag.step = s->step;
  return 0;
}

int or_step(or_sim* s, double dt, uint32_t nsteps) {
  for (uint32_t i = 0; i < nsteps; ++i) {
    if (or_transport(s, dt)) return -1;
    if (or_react(s, dt)) return -1;
  }
  return 0;
}

/* ---- dynamic time step ---------------------------------------------------------
 * The paper runs fixed steps and names CFL- or physics-based stepping as the next step
 * (section Final algorithm, closing paragraph).  Reading taken here: the step is the
 * smallest of
 *   dt_max,
 *   c_drift dx / v(Emax)          (drift CFL: no particle drifts more than c_drift cells),
 *   c_diff dx^2 / (2 D)           (no axis's diffusive spread exceeds sqrt(c_diff) cells),
 *   c_ion / (alpha(Emax) v(Emax)) (at most c_ion expected ionizations per electron),
 * with v(E) = mu(E) E and Emax the largest |E^k| over the cell centres (uniform mode:
 * |E_uniform|).  A CIC-interpolated field is a convex combination of cell-centre values,
 * so no particle sees a field above Emax; v and alpha v grow with E (mu_b >= -1), so
 * the limits hold for every particle.  A limit whose factor is <= 0, or whose rate is
 * zero, is not applied. */
double or_field_max(or_sim* s) {
  const or_desc* d = &s->d;
  if (d->field_mode == OR_FIELD_UNIFORM) {
    const double* E = d->E_uniform;
    return sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
  }
  if (!s->field_valid) initial_field(s);
  double m2 = 0.0;
  for (int64_t c = 0; c < s->ncell; ++c) {
    double e2 = s->Ex[c] * s->Ex[c] + s->Ey[c] * s->Ey[c] + s->Ez[c] * s->Ez[c];
    if (e2 > m2) m2 = e2;
  }
  return sqrt(m2);
}

double or_stable_dt(or_sim* s, const or_dt_rule* r, double* Emax_out) {
  const or_coeffs* c = &s->c;
  const double dx = s->d.dx;
  const double Em = or_field_max(s);
  if (Emax_out) *Emax_out = Em;
  double dt = r->dt_max;
  const double v = or_mobility(c, Em) * Em;
  if (r->c_drift > 0.0 && v > 0.0) dt = fmin(dt, r->c_drift * dx / v);
  if (r->c_diff > 0.0 && c->D > 0.0) dt = fmin(dt, r->c_diff * dx * dx / (2.0 * c->D));
  const double nu = Em > 0.0 ? c->alpha_A * exp(-c->alpha_B / Em) * v : 0.0;
  if (r->c_ion > 0.0 && nu > 0.0) dt = fmin(dt, r->c_ion / nu);
  return dt;
}

int or_step_adaptive(or_sim* s, const or_dt_rule* r, uint32_t nsteps, double* dts) {
  for (uint32_t i = 0; i < nsteps; ++i) {
    const double dt = or_stable_dt(s, r, NULL);
    if (dts) dts[i] = dt;
    if (or_transport(s, dt)) return -1;
    if (or_react(s, dt)) return -1;
  }
  return 0;
}

void or_diagnostics(const or_sim* s, or_diag* out) {
  *out = s->diag;
  out->n_particles = s->np;
  uint64_t W = 0;
  for (uint64_t i = 0; i < s->np; ++i) W += s->p[i].w;
  out->weight = W;
  int64_t P = 0, Mn = 0;
  for (int64_t c = 0; c < s->ncell; ++c) { P += s->nplus[c]; Mn += s->nminus[c]; }
  out->n_plus = P;
  out->n_minus = Mn;
  out->charge = P - (int64_t)W - Mn;
  out->step = s->step;
}
