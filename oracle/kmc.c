/*
 * Oracle: per-cell Kinetic Monte Carlo (test infrastructure; see oracle.h).
 *
 * Follows the paper's section "Kinetic Monte Carlo" (reaction network, propensities,
 * SSA, tau-leaping, eq. tau_leaping) and the eight-step hybrid outline of its
 * section "Reaction algorithm outline" (after Cao, Gillespie and Petzold), with the
 * paper's choices N_c = 5, N_SSA = 10 and the SSA exception when A * dtau <= 1.  The
 * network is the paper's air-chemistry table, over species (e, M+, M-, gamma):
 *   R1  e -> e + e + M+   (k_alpha)   a = k X_e        nu = (+1, +1,  0,  0)
 *   R2  e -> M-           (k_eta)     a = k X_e        nu = (-1,  0, +1,  0)
 *   R3  e -> e + gamma    (k_gamma)   a = k X_e        nu = ( 0,  0,  0, +1)
 *   R4  e + M+ -> 0       (k_ep)      a = k X_e X_M+   nu = (-1, -1,  0,  0)
 *   R5  M- + M+ -> 0      (k_np)      a = k X_M+ X_M-  nu = ( 0, -1, -1,  0)
 * (the table's rows 1, 2, 5, 3 and 4).  A reaction belongs to a cell's network when its
 * rate constant there is positive; with k_ep = k_np = 0 the network is the three
 * first-order reactions the paper's example simulations use.
 *
 * Readings where the text is silent:
 *   - step 4's factor g_i follows Cao, Gillespie and Petzold (2006): 1 when the highest
 *     order of a network reaction that consumes species i as a reactant is one, 2 when
 *     it is a second-order reaction between two different species (R4, R5); the paper
 *     uses g_i = 1 because its examples are first order;
 *   - a rejected leap halves the attempted step: dtau_nc := dtau / 2 (with eps = inf
 *     halving "infinity" has no meaning);
 *   - the SSA exception (A dtau <= 1, dtau = min(dt - tau, dtau_nc)) is tested before
 *     the critical time of step 3 is drawn, as in the algorithm of Cao, Gillespie and
 *     Petzold (2006) that the paper defers to: taken in the printed order, the SSA of
 *     branch 6(b) would give critical reactions a second chance to fire after step 3
 *     has already found that they do not, doubling their rate in the SSA limit.  The
 *     excursion advances tau by the time of at most N_SSA events, or by all of dtau if
 *     the next event falls beyond it;
 *   - a critical reaction is a network reaction with a consumed reactant i (nu_ri < 0)
 *     for which X_i < N_c |nu_ri| (a reactant that five firings would exhaust);
 *   - a selection by u takes the first reaction, in table order, whose cumulative
 *     propensity exceeds u times the total, and the last one with a positive propensity
 *     if rounding leaves none;
 *   - uniform draws come from the cell's sequential Philox stream (cell, step, KMC);
 *     a logarithm always takes a draw in (0,1], a selection a draw in [0,1).
 * Pins (tests): Poisson-distributed one-leap counts in pure tau-leap mode; the linear
 * birth-death extinction probability; mean growth exp((k_alpha - k_eta) t) and the
 * discrete form (1 + (k_alpha - k_eta) dt)^K; the exact laws of the two recombination
 * death chains (master equation); the leap bound's relative propensity change against
 * eps; charge conservation; non-negativity.
 */
#include "or_internal.h"

#define NS 4
#define NR 5
static const int NU[NR][NS] = {
  {+1, +1, 0, 0},   /* ionization            */
  {-1, 0, +1, 0},   /* attachment            */
  {0, 0, 0, +1},    /* photon emission       */
  {-1, -1, 0, 0},   /* electron-ion recombination */
  {0, -1, -1, 0},   /* ion-ion recombination */
};
/* reactants of each reaction: species indices, -1 for none */
static const int REACT[NR][2] = {{0, -1}, {0, -1}, {0, -1}, {0, 1}, {1, 2}};

static void propensities(const int64_t X[NS], const double k[NR], double a[NR]) {
  for (int r = 0; r < NR; ++r) {
    double v = k[r] * (double)X[REACT[r][0]];
    if (REACT[r][1] >= 0) v *= (double)X[REACT[r][1]];
    a[r] = v;
  }
}

static double total(const double a[NR]) {
  double A = 0.0;
  for (int r = 0; r < NR; ++r) A += a[r];
  return A;
}

static int is_critical(const or_desc* d, const int64_t X[NS], const double k[NR], int r) {
  if (!(k[r] > 0.0)) return 0;
  for (int i = 0; i < NS; ++i)
    if (NU[r][i] < 0 && X[i] < (int64_t)d->kmc_nc * (int64_t)(-NU[r][i])) return 1;
  return 0;
}

/* first selected reaction with cumsum_{r<=j} a_r > u * sum; the last selected one with a
 * positive propensity if rounding leaves none */
static int select_reaction(const double a[NR], const int use[NR], double sum, double u) {
  double target = u * sum, acc = 0.0;
  int last = -1;
  for (int r = 0; r < NR; ++r) {
    if (!use[r]) continue;
    acc += a[r];
    if (a[r] > 0.0) last = r;
    if (acc > target) return r;
  }
  return last;
}

/* g_i of step 4: the highest order of a network reaction with species i as reactant */
static double g_factor(const double k[NR], int i) {
  int order = 1;
  for (int r = 0; r < NR; ++r) {
    if (!(k[r] > 0.0)) continue;
    int n = REACT[r][1] >= 0 ? 2 : 1;
    if ((REACT[r][0] == i || REACT[r][1] == i) && n > order) order = n;
  }
  return (double)order;
}

static double tau_nc_bound(const or_desc* d, const int64_t X[NS], const double k[NR],
                           const double a[NR], const int crit[NR]) {
  if (isinf(d->kmc_eps)) return INFINITY;
  double best = INFINITY;
  for (int i = 0; i < NS; ++i) {
    int reactant = 0;
    for (int r = 0; r < NR; ++r)
      if (k[r] > 0.0 && !crit[r] && (REACT[r][0] == i || REACT[r][1] == i)) reactant = 1;
    if (!reactant) continue;
    double mu = 0.0, var = 0.0;
    for (int r = 0; r < NR; ++r) {
      if (!(k[r] > 0.0) || crit[r]) continue;
      mu += NU[r][i] * a[r];
      var += (double)NU[r][i] * NU[r][i] * a[r];
    }
    double bound = fmax(d->kmc_eps * (double)X[i] / g_factor(k, i), 1.0);
    if (mu != 0.0) best = fmin(best, bound / fabs(mu));
    if (var > 0.0) best = fmin(best, bound * bound / var);
  }
  return best;
}

double or_kmc_leap_bound(const or_desc* d, const int64_t X[4], const double k[5]) {
  double a[NR];
  int crit[NR];
  propensities(X, k, a);
  for (int r = 0; r < NR; ++r) crit[r] = is_critical(d, X, k, r);
  return tau_nc_bound(d, X, k, a, crit);
}

/* One SSA excursion over the whole network: at most N_SSA events within h.
 * Returns the time advanced (h if the next event falls beyond h). */
static double ssa_excursion(const or_desc* d, int64_t X[NS], const double k[NR], double h,
                            or_stream* s, int64_t fires[NR]) {
  double a[NR], tp = 0.0;
  int all[NR] = {1, 1, 1, 1, 1};
  propensities(X, k, a);
  double A = total(a);
  for (int events = 0; events < d->kmc_nssa; ++events) {
    if (!(A > 0.0)) return h;
    double delta = log(1.0 / or_u_oc(or_stream_next(s))) / A;
    if (tp + delta > h) return h;
    int j = select_reaction(a, all, A, or_u_co(or_stream_next(s)));
    for (int i = 0; i < NS; ++i) X[i] += NU[j][i];
    fires[j] += 1;
    tp += delta;
    propensities(X, k, a);
    A = total(a);
  }
  return tp;
}

static void kmc_hybrid(const or_desc* d, int64_t X[NS], const double k[NR], double dt,
                       or_stream* s, int64_t fires[NR]) {
  double tau = 0.0;
  while (tau < dt) {
    /* steps 1-2: critical set and propensities */
    double a[NR];
    int crit[NR], ncrit[NR];
    propensities(X, k, a);
    double A = 0.0, Ac = 0.0;
    for (int r = 0; r < NR; ++r) {
      A += a[r];
      crit[r] = is_critical(d, X, k, r);
      ncrit[r] = !crit[r];
      if (crit[r]) Ac += a[r];
    }
    if (!(A > 0.0)) break;                      /* nothing can fire any more */
    /* step 4: non-critical leap bound */
    double dtnc = tau_nc_bound(d, X, k, a, crit);
    double dtc = INFINITY;
    int have_dtc = 0;
    for (;;) {
      double rem = dt - tau;
      double h = fmin(rem, dtnc);
      /* SSA exception, tested before the critical time is drawn (ordering of Cao et
       * al. 2006): the SSA then handles critical reactions itself */
      if (A * h <= 1.0) {
        double tp = ssa_excursion(d, X, k, h, s, fires);
        tau = (tp == rem) ? dt : tau + tp;     /* consuming the remainder ends the step */
        break;                                  /* back to step 1 */
      }
      /* step 3: time to the next critical reaction, drawn once per step-1 pass */
      if (!have_dtc) {
        if (Ac > 0.0) dtc = log(1.0 / or_u_oc(or_stream_next(s))) / Ac;
        have_dtc = 1;
      }
      /* step 5 */
      double dtau = fmin(h, dtc);
      int64_t Xn[NS], f[NR] = {0, 0, 0, 0, 0};
      memcpy(Xn, X, sizeof(Xn));
      if (dtc < dtnc && dtc < rem) {
        /* 6(a): one critical reaction plus Poisson firings of the non-critical ones */
        int rc = select_reaction(a, crit, Ac, or_u_co(or_stream_next(s)));
        f[rc] += 1;
        for (int i = 0; i < NS; ++i) Xn[i] += NU[rc][i];
      }
      /* 6(a)/(b): non-critical reactions by tau-leaping over dtau */
      for (int r = 0; r < NR; ++r) {
        if (!ncrit[r]) continue;
        int64_t n = or_poisson(a[r] * dtau, s);
        f[r] += n;
        for (int i = 0; i < NS; ++i) Xn[i] += n * NU[r][i];
      }
      int bad = 0;
      for (int i = 0; i < NS; ++i) if (Xn[i] < 0) bad = 1;
      if (bad) { dtnc = dtau / 2.0; continue; }   /* step 7(a): reject, halve, retry */
      memcpy(X, Xn, sizeof(Xn));
      for (int r = 0; r < NR; ++r) fires[r] += f[r];
      tau = (dtau == rem) ? dt : tau + dtau;
      break;
    }
  }
}

/* Pure tau-leaping (eq. tau_leaping) over dt; a leap that would make a population
 * negative is rejected and retried with half the step. */
static void kmc_pure_tau(int64_t X[NS], const double k[NR], double dt, or_stream* s,
                         int64_t fires[NR]) {
  double tau = 0.0, hmax = INFINITY;
  while (tau < dt) {
    double a[NR];
    propensities(X, k, a);
    if (!(total(a) > 0.0)) break;
    double h = fmin(dt - tau, hmax);
    int64_t Xn[NS], f[NR];
    memcpy(Xn, X, sizeof(Xn));
    for (int r = 0; r < NR; ++r) {
      f[r] = or_poisson(a[r] * h, s);
      for (int i = 0; i < NS; ++i) Xn[i] += f[r] * NU[r][i];
    }
    int bad = 0;
    for (int i = 0; i < NS; ++i) if (Xn[i] < 0) bad = 1;
    if (bad) { hmax = h / 2.0; continue; }
    memcpy(X, Xn, sizeof(Xn));
    for (int r = 0; r < NR; ++r) fires[r] += f[r];
    tau = (h == dt - tau) ? dt : tau + h;
  }
}

void or_kmc_advance(const or_desc* d, int64_t X[4], const double k[5], double dt,
                    or_stream* s, int64_t fires[5]) {
  for (int r = 0; r < NR; ++r) fires[r] = 0;
  if (d->kmc_mode == OR_KMC_PURE_TAU) kmc_pure_tau(X, k, dt, s, fires);
  else kmc_hybrid(d, X, k, dt, s, fires);
}

void or_kmc_cells(const or_desc* d, int64_t n_cells, const uint32_t* cell_ids, int64_t* X,
                  const double* k, double dt, uint32_t step, int64_t* fires) {
  for (int64_t c = 0; c < n_cells; ++c) {
    or_stream s;
    or_stream_init(&s, cell_ids[c], step, OR_TAG_KMC, 0, d->seed, d->realization);
    or_kmc_advance(d, X + 4 * c, k + 5 * c, dt, &s, fires + 5 * c);
  }
}
