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
    if (a1 > target) { X.e += 1; X.p += 1; f[0] += 1; }
    else if (a1 + a2 > target) { X.e -= 1; X.m += 1; f[1] += 1; }
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


}  // namespace itk
