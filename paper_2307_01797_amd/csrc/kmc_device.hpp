// Per-cell Kinetic Monte Carlo device code shared by the single-realization and the
// ensemble kernels (see kmc.hip for the method and its readings).
#pragma once
#include <math.h>

#include "device.hpp"
#include "poisson.hpp"

namespace itk {

struct KmcParams {
  int mode, nc, nssa;
  double eps;
};

struct State {
  int64_t e, p, m, g;
};

// Largest leap that keeps the relative change of the non-critical propensities below
// eps (step 4, g_i = 1); infinite for eps = inf.
__device__ inline double leap_bound(const KmcParams& P, const State& X, double a1, double a2,
                             double a3, bool crit2) {
  if (isinf(P.eps)) return INFINITY;
  // the only reactant is e; net and squared changes of e over non-critical reactions
  double mu = 0.0 + 1.0 * a1;
  double var = 0.0 + 1.0 * a1;
  if (!crit2) { mu = mu + (-1.0) * a2; var = var + 1.0 * a2; }
  mu = mu + 0.0 * a3;
  var = var + 0.0 * a3;
  const double bound = fmax(P.eps * (double)X.e / 1.0, 1.0);
  double best = INFINITY;
  if (mu != 0.0) best = fmin(best, bound / fabs(mu));
  if (var > 0.0) best = fmin(best, bound * bound / var);
  return best;
}

// Whole-network SSA for at most nssa events inside h; returns the time advanced.
__device__ inline double ssa_run(const KmcParams& P, State& X, const double k[3], double h,
                          CellStream& st, int64_t f[3]) {
  double tp = 0.0;
#pragma unroll 1
  for (int ev = 0; ev < P.nssa; ++ev) {
    const double a1 = k[0] * (double)X.e, a2 = k[1] * (double)X.e, a3 = k[2] * (double)X.e;
    const double A = a1 + a2 + a3;
    if (!(A > 0.0)) return h;
    const double delta = log(1.0 / u_oc(st.next())) / A;
    if (tp + delta > h) return h;
    const double target = u_co(st.next()) * A;
    // the first reaction whose cumulative propensity exceeds u A; if rounding leaves
    // none, the last one with a positive propensity
    const int j = a1 > target ? 0 : (a1 + a2 > target ? 1 : (a1 + a2 + a3 > target || a3 > 0.0 ? 2 : (a2 > 0.0 ? 1 : 0)));
    if (j == 0) { X.e += 1; X.p += 1; f[0] += 1; }
    else if (j == 1) { X.e -= 1; X.m += 1; f[1] += 1; }
    else { X.g += 1; f[2] += 1; }
    tp += delta;
  }
  return tp;
}

__device__ inline void advance_hybrid(const KmcParams& P, State& X, const double k[3], double dt,
                               CellStream& st, int64_t f[3]) {
  double tau = 0.0;
  for (int pass = 0; tau < dt && pass < (1 << 22); ++pass) {  // bounded: every pass fires or advances
    const double a1 = k[0] * (double)X.e, a2 = k[1] * (double)X.e, a3 = k[2] * (double)X.e;
    const double A = a1 + a2 + a3;
    if (!(A > 0.0)) break;
    const bool crit2 = (a2 > 0.0) && X.e < (int64_t)P.nc;
    const double Ac = crit2 ? a2 : 0.0;
    double dtnc = leap_bound(P, X, a1, a2, a3, crit2);
    double dtc = INFINITY;
    bool drawn = false;
    for (int attempt = 0; attempt < 4096; ++attempt) {
      const double rem = dt - tau;
      const double h = fmin(rem, dtnc);
      if (A * h <= 1.0) {
        const double tp = ssa_run(P, X, k, h, st, f);
        tau = (tp == rem) ? dt : tau + tp;
        break;
      }
      if (!drawn) {
        if (Ac > 0.0) dtc = log(1.0 / u_oc(st.next())) / Ac;
        drawn = true;
      }
      const double dtau = fmin(h, dtc);
      State Y = X;
      int64_t g[3] = {0, 0, 0};
      if (dtc < dtnc && dtc < rem) {
        (void)st.next();            // selection among the critical set (attachment only)
        Y.e -= 1; Y.m += 1; g[1] += 1;
      }
      // non-critical reactions leap over dtau, in table order
      const int64_t n1 = poisson_draw(a1 * dtau, st);
      Y.e += n1; Y.p += n1; g[0] += n1;
      if (!crit2) {
        const int64_t n2 = poisson_draw(a2 * dtau, st);
        Y.e -= n2; Y.m += n2; g[1] += n2;
      }
      const int64_t n3 = poisson_draw(a3 * dtau, st);
      Y.g += n3; g[2] += n3;
      if (Y.e < 0 || Y.p < 0 || Y.m < 0 || Y.g < 0) { dtnc = dtau / 2.0; continue; }
      X = Y;
      f[0] += g[0]; f[1] += g[1]; f[2] += g[2];
      tau = (dtau == rem) ? dt : tau + dtau;
      break;
    }
  }
}

__device__ inline void advance_pure_tau(State& X, const double k[3], double dt, CellStream& st,
                                 int64_t f[3]) {
  double tau = 0.0, hmax = INFINITY;
  for (int it = 0; tau < dt && it < 100000; ++it) {
    const double a1 = k[0] * (double)X.e, a2 = k[1] * (double)X.e, a3 = k[2] * (double)X.e;
    if (!(a1 + a2 + a3 > 0.0)) break;
    const double h = fmin(dt - tau, hmax);
    const int64_t n1 = poisson_draw(a1 * h, st);
    const int64_t n2 = poisson_draw(a2 * h, st);
    const int64_t n3 = poisson_draw(a3 * h, st);
    State Y = X;
    Y.e += n1 - n2; Y.p += n1; Y.m += n2; Y.g += n3;
    if (Y.e < 0) { hmax = h / 2.0; continue; }
    X = Y;
    f[0] += n1; f[1] += n2; f[2] += n3;
    tau = (h == dt - tau) ? dt : tau + h;
  }
}

// The common case of the hybrid method, with a small register footprint: the whole step
// is one SSA excursion (A h <= 1 for h = dt, i.e. no leap bound below dt) that ends at
// dt within nssa events, or nothing can fire (A = 0).  Then X, f and the stream are
// exactly what advance() produces and the result is true.  Otherwise false: the caller
// discards X, f and the stream and runs advance() from the original state.
__device__ __forceinline__ bool advance_fast(const KmcParams& P, State& X, const double k[3],
                                             double dt, CellStream& st, int64_t f[3]) {
  f[0] = f[1] = f[2] = 0;
  if (P.mode != ITOKMC_KMC_HYBRID) return false;
  const double a1 = k[0] * (double)X.e, a2 = k[1] * (double)X.e, a3 = k[2] * (double)X.e;
  const double A = a1 + a2 + a3;
  if (!(A > 0.0)) return true;
  const bool crit2 = (a2 > 0.0) && X.e < (int64_t)P.nc;
  const double h = fmin(dt, leap_bound(P, X, a1, a2, a3, crit2));
  if (h != dt || !(A * h <= 1.0)) return false;
  return ssa_run(P, X, k, h, st, f) == dt;
}

__device__ __forceinline__ void advance(const KmcParams& P, State& X, const double k[3], double dt,
                                        CellStream& st, int64_t f[3]) {
  f[0] = f[1] = f[2] = 0;
  if (P.mode == ITOKMC_KMC_PURE_TAU) advance_pure_tau(X, k, dt, st, f);
  else advance_hybrid(P, X, k, dt, st, f);
}

// ---- the network with recombination ------------------------------------------------
// Five reactions over (e, M+, M-, photons), in table order: ionization, attachment,
// photo-emission (first order in e), electron-ion recombination e + M+ (a = k X_e X_M+)
// and ion-ion recombination M- + M+ (a = k X_M+ X_M-).  A reaction is part of a cell's
// network when its rate is positive.  The steps are those of the three-reaction code
// above, written over the reaction table: critical reactions are network reactions a
// few firings from exhausting a reactant; the leap bound of step 4 takes g_i = 2 for a
// species consumed by a second-order reaction of the network (Cao, Gillespie and
// Petzold 2006), 1 otherwise.

__host__ __device__ constexpr int nu5(int r, int i) {
  return r == 0 ? ((i == 0 || i == 1) ? 1 : 0)
       : r == 1 ? (i == 0 ? -1 : (i == 2 ? 1 : 0))
       : r == 2 ? (i == 3 ? 1 : 0)
       : r == 3 ? ((i == 0 || i == 1) ? -1 : 0)
       : ((i == 1 || i == 2) ? -1 : 0);
}
__host__ __device__ constexpr bool reactant5(int r, int i) {
  return r < 3 ? i == 0 : (r == 3 ? (i == 0 || i == 1) : (i == 1 || i == 2));
}

struct State5 {
  int64_t x[4];
};

__device__ __forceinline__ void props5(const State5& X, const double k[5], double a[5]) {
  a[0] = k[0] * (double)X.x[0];
  a[1] = k[1] * (double)X.x[0];
  a[2] = k[2] * (double)X.x[0];
  a[3] = k[3] * (double)X.x[0] * (double)X.x[1];
  a[4] = k[4] * (double)X.x[1] * (double)X.x[2];
}

__device__ __forceinline__ void fire5(State5& X, int r, int64_t n) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
#pragma unroll
    for (int q = 0; q < 5; ++q)
      if (q == r) X.x[i] += n * (int64_t)nu5(q, i);
  }
}

__device__ __forceinline__ bool critical5(const KmcParams& P, const State5& X, const double k[5], int r) {
  if (!(k[r] > 0.0)) return false;
  bool c = false;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (nu5(r, i) < 0 && X.x[i] < (int64_t)P.nc * (int64_t)(-nu5(r, i))) c = true;
  return c;
}

// first selected reaction with cumulative propensity above u * sum, else the last
// selected one with a positive propensity
__device__ __forceinline__ int select5(const double a[5], const bool use[5], double sum, double u) {
  const double target = u * sum;
  double acc = 0.0;
  int last = -1;
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    if (!use[r]) continue;
    acc += a[r];
    if (a[r] > 0.0) last = r;
    if (acc > target) return r;
  }
  return last;
}

__device__ inline double leap_bound5(const KmcParams& P, const State5& X, const double k[5],
                                     const double a[5], const bool crit[5]) {
  if (isinf(P.eps)) return INFINITY;
  double best = INFINITY;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    bool reactant = false;
    double g = 1.0;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      if (k[r] > 0.0 && !crit[r] && reactant5(r, i)) reactant = true;
      if (k[r] > 0.0 && reactant5(r, i) && r >= 3) g = 2.0;
    }
    if (!reactant) continue;
    double mu = 0.0, var = 0.0;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      if (!(k[r] > 0.0) || crit[r]) continue;
      mu += (double)nu5(r, i) * a[r];
      var += (double)nu5(r, i) * (double)nu5(r, i) * a[r];
    }
    const double bound = fmax(P.eps * (double)X.x[i] / g, 1.0);
    if (mu != 0.0) best = fmin(best, bound / fabs(mu));
    if (var > 0.0) best = fmin(best, bound * bound / var);
  }
  return best;
}

__device__ inline double ssa_run5(const KmcParams& P, State5& X, const double k[5], double h,
                                  CellStream& st, int64_t f[5]) {
  const bool all[5] = {true, true, true, true, true};
  double tp = 0.0;
#pragma unroll 1
  for (int ev = 0; ev < P.nssa; ++ev) {
    double a[5];
    props5(X, k, a);
    const double A = a[0] + a[1] + a[2] + a[3] + a[4];
    if (!(A > 0.0)) return h;
    const double delta = log(1.0 / u_oc(st.next())) / A;
    if (tp + delta > h) return h;
    const int j = select5(a, all, A, u_co(st.next()));
    fire5(X, j, 1);
    f[j] += 1;
    tp += delta;
  }
  return tp;
}

__device__ inline void advance_hybrid5(const KmcParams& P, State5& X, const double k[5], double dt,
                                       CellStream& st, int64_t f[5]) {
  double tau = 0.0;
  for (int pass = 0; tau < dt && pass < (1 << 22); ++pass) {  // bounded: every pass fires or advances
    double a[5];
    bool crit[5], ncrit[5];
    props5(X, k, a);
    double A = 0.0, Ac = 0.0;
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      A += a[r];
      crit[r] = critical5(P, X, k, r);
      ncrit[r] = !crit[r];
      if (crit[r]) Ac += a[r];
    }
    if (!(A > 0.0)) break;
    double dtnc = leap_bound5(P, X, k, a, crit);
    double dtc = INFINITY;
    bool drawn = false;
    for (int attempt = 0; attempt < 4096; ++attempt) {
      const double rem = dt - tau;
      const double h = fmin(rem, dtnc);
      if (A * h <= 1.0) {
        const double tp = ssa_run5(P, X, k, h, st, f);
        tau = (tp == rem) ? dt : tau + tp;
        break;
      }
      if (!drawn) {
        if (Ac > 0.0) dtc = log(1.0 / u_oc(st.next())) / Ac;
        drawn = true;
      }
      const double dtau = fmin(h, dtc);
      State5 Y = X;
      int64_t g[5] = {0, 0, 0, 0, 0};
      if (dtc < dtnc && dtc < rem) {
        const int rc = select5(a, crit, Ac, u_co(st.next()));
        g[rc] += 1;
        fire5(Y, rc, 1);
      }
#pragma unroll
      for (int r = 0; r < 5; ++r) {
        if (!ncrit[r]) continue;
        const int64_t n = poisson_draw(a[r] * dtau, st);
        g[r] += n;
        fire5(Y, r, n);
      }
      if (Y.x[0] < 0 || Y.x[1] < 0 || Y.x[2] < 0 || Y.x[3] < 0) { dtnc = dtau / 2.0; continue; }
      X = Y;
#pragma unroll
      for (int r = 0; r < 5; ++r) f[r] += g[r];
      tau = (dtau == rem) ? dt : tau + dtau;
      break;
    }
  }
}

__device__ inline void advance_pure_tau5(State5& X, const double k[5], double dt, CellStream& st,
                                         int64_t f[5]) {
  double tau = 0.0, hmax = INFINITY;
  for (int it = 0; tau < dt && it < 100000; ++it) {
    double a[5];
    props5(X, k, a);
    if (!(a[0] + a[1] + a[2] + a[3] + a[4] > 0.0)) break;
    const double h = fmin(dt - tau, hmax);
    State5 Y = X;
    int64_t g[5];
#pragma unroll
    for (int r = 0; r < 5; ++r) {
      g[r] = poisson_draw(a[r] * h, st);
      fire5(Y, r, g[r]);
    }
    if (Y.x[0] < 0 || Y.x[1] < 0 || Y.x[2] < 0 || Y.x[3] < 0) { hmax = h / 2.0; continue; }
    X = Y;
#pragma unroll
    for (int r = 0; r < 5; ++r) f[r] += g[r];
    tau = (h == dt - tau) ? dt : tau + h;
  }
}

__device__ __forceinline__ void advance5(const KmcParams& P, State5& X, const double k[5], double dt,
                                         CellStream& st, int64_t f[5]) {
#pragma unroll
  for (int r = 0; r < 5; ++r) f[r] = 0;
  if (P.mode == ITOKMC_KMC_PURE_TAU) advance_pure_tau5(X, k, dt, st, f);
  else advance_hybrid5(P, X, k, dt, st, f);
}


}  // namespace itk
