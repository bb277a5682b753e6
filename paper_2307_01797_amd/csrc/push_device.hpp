// Per-particle Ito push arithmetic shared by the single-realization and the ensemble
// kernels: Philox normals and the Euler-Maruyama update in cell-relative offsets.
#pragma once
#include <math.h>

#include "device.hpp"

namespace itk {

template <typename T> struct Normals;
template <> struct Normals<double> {
  // Box-Muller on one Philox block; the fourth word's partner is unused.
  __device__ static void get(uint4 r, double n[3]) {
    const double two_pi = 6.283185307179586476925286766559;
    const double r0 = sqrt(-2.0 * log(u_oc(r.x)));
    const double t0 = two_pi * u_co(r.y);
    const double r1 = sqrt(-2.0 * log(u_oc(r.z)));
    const double t1 = two_pi * u_co(r.w);
    n[0] = r0 * cos(t0);
    n[1] = r0 * sin(t0);
    n[2] = r1 * cos(t1);
  }
};
template <> struct Normals<float> {
  // Single precision: hardware log2 and sin/cos of revolutions (v_log_f32, v_sin_f32,
  // v_cos_f32); -2 ln u = -2 ln2 log2 u.
  __device__ static void get(uint4 r, float n[3]) {
    const float m2ln2 = -1.3862943611198906f;
    const float r0 = __builtin_sqrtf(m2ln2 * __builtin_amdgcn_logf(u_ocf(r.x)));
    const float r1 = __builtin_sqrtf(m2ln2 * __builtin_amdgcn_logf(u_ocf(r.z)));
    const float a0 = (float)(r.y >> 8) * 0x1p-24f;
    const float a1 = (float)(r.w >> 8) * 0x1p-24f;
    n[0] = r0 * __builtin_amdgcn_cosf(a0);
    n[1] = r0 * __builtin_amdgcn_sinf(a0);
    n[2] = r1 * __builtin_amdgcn_cosf(a1);
  }
};

// Advance one particle by drift + diff * N in grid units; returns false if it left
// the grid.  ci: cell indices in/out, o: offsets in [0,1) in/out.
template <typename T>
__device__ __forceinline__ bool push_uniform(uint64_t id, uint32_t step, Key key, const T drift[3],
                                             T diff, const int lim[3], int ci[3], T o[3]) {
  const uint4 r = philox_block((uint32_t)id, (uint32_t)(id >> 32), step, TAG_PUSH, 0, key);
  T nr[3];
  Normals<T>::get(r, nr);
  bool inside = true;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    T x = o[ax] + (drift[ax] + diff * nr[ax]);
    T f = floor(x);
    x -= f;
    if (x >= (T)1) { x -= (T)1; f += (T)1; }
    o[ax] = x;
    ci[ax] += (int)f;
    inside = inside && ci[ax] >= 0 && ci[ax] < lim[ax];
  }
  return inside;
}

// Offset in [0,1) of the working precision.
template <typename T> __device__ __forceinline__ T to_off(double o);
template <> __device__ __forceinline__ double to_off<double>(double o) { return o; }
template <> __device__ __forceinline__ float to_off<float>(double o) {
  float f = (float)o;
  return f < 1.0f ? f : 0x1.fffffep-1f;
}

// Position in grid units of the i-th Gaussian seed electron (centre c and width sigma
// in metres, Box-Muller on the Philox block (i, SEED)); false if it falls outside.
__device__ inline bool gaussian_seed_point(uint64_t i, Key key, double dx, const int lim[3],
                                           const double c[3], double sigma, double xi[3]) {
  const double two_pi = 6.283185307179586476925286766559;
  const uint4 r = philox_block((uint32_t)i, (uint32_t)(i >> 32), 0, TAG_SEED, 0, key);
  const double r0 = sqrt(-2.0 * log(u_oc(r.x)));
  const double t0 = two_pi * u_co(r.y);
  const double r1 = sqrt(-2.0 * log(u_oc(r.z)));
  const double t1 = two_pi * u_co(r.w);
  const double nrm[3] = {r0 * cos(t0), r0 * sin(t0), r1 * cos(t1)};
  for (int a = 0; a < 3; ++a) xi[a] = (c[a] + sigma * nrm[a]) / dx;
  return xi[0] >= 0.0 && xi[0] < lim[0] && xi[1] >= 0.0 && xi[1] < lim[1] && xi[2] >= 0.0 &&
         xi[2] < lim[2];
}

}  // namespace itk
