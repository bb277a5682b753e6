// Poisson deviates on the device, drawn from a cell's sequential stream: sequential
// CDF inversion (one uniform in [0,1)) for means below 10, and the transformed
// rejection method PTRS of Hormann (1993) for larger means (two uniforms per trial).
// A mean <= 0 returns 0 without consuming a draw.  All arithmetic in double.
#pragma once
#include "device.hpp"

namespace itk {

// Mean in (0, 10): sequential CDF inversion.
__device__ inline int64_t poisson_small(double lam, CellStream& st) {
  const double u = u_co(st.next());
  double term = exp(-lam);
  double cdf = term;
  int64_t k = 0;
  while (u >= cdf && k < 1000) {
    ++k;
    term *= lam / (double)k;
    cdf += term;
  }
  return k;
}

// Mean >= 10: PTRS.
__device__ inline int64_t poisson_ptrs(double lam, CellStream& st) {
  const double sl = sqrt(lam);
  const double ll = log(lam);
  const double b = 0.931 + 2.53 * sl;
  const double a = -0.059 + 0.02483 * b;
  const double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  const double v_r = 0.9277 - 3.6224 / (b - 2.0);
  for (int trial = 0; trial < 100000; ++trial) {
    const double U = u_co(st.next()) - 0.5;
    const double V = u_oc(st.next());
    const double us = 0.5 - fabs(U);
    const double kd = floor((2.0 * a / us + b) * U + lam + 0.43);
    if (us >= 0.07 && V <= v_r) return (int64_t)kd;
    if (kd < 0.0 || (us < 0.013 && V > us)) continue;
    const double lhs = log(V) + log(inv_alpha) - log(a / (us * us) + b);
    const double rhs = -lam + kd * ll - lgamma(kd + 1.0);
    if (lhs <= rhs) return (int64_t)kd;
  }
  return (int64_t)floor(lam);  // unreachable in practice; bounds the loop
}

__device__ inline int64_t poisson_draw(double lam, CellStream& st) {
  if (!(lam > 0.0)) return 0;
  return lam < 10.0 ? poisson_small(lam, st) : poisson_ptrs(lam, st);
}

}  // namespace itk
