// Self-consistent field mode: the semi-implicit Euler-Maruyama step of the paper's
// "Final algorithm" (steps 1-5) and its field solve.
//
//   1. sigma^k = e sum_p mu_p w_p W(x - X_p^k) / dV with mu_p = mu(|E^k(X_p^k)|)
//      (eq. conductivity, electrons only; ions are immobile);
//   2. X_dagger = X^k + sqrt(2 D dt) N, regenerated from the particle's push stream;
//   3. rho_dagger = e (n+ - n- - CIC(X_dagger)) / dV, solve
//      div[(1 + sigma dt / eps0) grad phi] = -rho_dagger / eps0 (eq. poisson_simp) with
//      phi = 0 at z = 0, phi = V at z = L, homogeneous Neumann on x and y;
//   4-5. X^{k+1} = X_dagger - mu_p E^{k+1}(X^k) dt, binned by cell as in the uniform push.
//
// Discretisation: cell-centred finite volumes, 7-point stencil, face coefficients the
// harmonic mean of the two cell values, a Dirichlet face using the cell's own value
// over half a cell; E at cell centres by central differences with ghost values from
// the same conditions; CIC deposit/interpolation with tent weights about cell centres,
// clouds folded into the wall cells.
//
// Solver: geometric multigrid V(2,2) cycles with red-black Gauss-Seidel, cell-averaged
// restriction and trilinear prolongation, run in the working precision on the
// correction equation of an iterative-refinement loop whose residual and potential
// are kept in double; the loop stops at ||r||_2 <= rtol ||b||_2 (the paper's relative
// multigrid tolerance, 1e-10 by default).
#include <math.h>

#include <vector>


#include "device.hpp"
#include "itk.hpp"

namespace itk {

namespace {

constexpr double kE = 1.602176634e-19;
constexpr double kEps0 = 8.8541878128e-12;
constexpr int kMaxLevels = 12;
constexpr int kBottomMaxCells = 4096;

struct Level {
  int nx, ny, nz;
  uint32_t n;
  void* u;    // correction
  void* f;    // right-hand side (scaled by h^2)
  void* eps;  // cell coefficient 1 + sigma dt / eps0
};

struct Coef {
  double mu_a, mu_E0, mu_b, E_floor, D;
};

template <typename T>
__device__ __forceinline__ T* tp(void* p) { return reinterpret_cast<T*>(p); }
template <typename T>
__device__ __forceinline__ const T* ctp(const void* p) { return reinterpret_cast<const T*>(p); }

// Four values of T as one 16- (float) or two 16-byte (double) accesses.
template <typename T>
struct V4 {
  T a[4];
};

template <typename T>
__device__ __forceinline__ V4<T> ld4(const T* p) {
  V4<T> v;
  if constexpr (sizeof(T) == 4) {
    const float4 x = *reinterpret_cast<const float4*>(p);
    v.a[0] = x.x; v.a[1] = x.y; v.a[2] = x.z; v.a[3] = x.w;
  } else {
    const double2 x = reinterpret_cast<const double2*>(p)[0], y = reinterpret_cast<const double2*>(p)[1];
    v.a[0] = x.x; v.a[1] = x.y; v.a[2] = y.x; v.a[3] = y.y;
  }
  return v;
}

template <typename T>
__device__ __forceinline__ void st4(T* p, const T a0, const T a1, const T a2, const T a3) {
  if constexpr (sizeof(T) == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(a0, a1, a2, a3);
  } else {
    reinterpret_cast<double2*>(p)[0] = make_double2(a0, a1);
    reinterpret_cast<double2*>(p)[1] = make_double2(a2, a3);
  }
}


constexpr int kRedBlocks = 1024;  // fixed grid of the norm kernels: one partial per block

// Block-wide sum of a double (256 threads), valid in thread 0.
__device__ __forceinline__ double block_sumd(double v) {
  __shared__ double sh[4];
  v = wave_sumd(v);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = sh[0] + sh[1] + sh[2] + sh[3];
  __syncthreads();
  return s;
}

// Sum of the per-block partials in a fixed order (deterministic).
__global__ void __launch_bounds__(1024) k_sum_partials(const double* part, int n, double* out) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) v += part[i];
  v = wave_sumd(v);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += sh[i];
    *out = s;
  }
}

// The residual's norm as k_sum_partials computes it, also written with ||b||^2 into
// mapped host memory, followed by a sequence number (after a system-scope fence), so
// that the host can wait for it by polling instead of a copy and a stream
// synchronisation.
__global__ void __launch_bounds__(1024) k_sum_notify(const double* part, int n, double* out,
                                                     const double* bn2, double* host,
                                                     unsigned long long* seq) {
  __shared__ double sh[16];
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) v += part[i];
  v = wave_sumd(v);
  if (lane_id() == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += sh[i];
    *out = s;
    host[0] = *bn2;
    host[1] = s;
    __threadfence_system();
    const unsigned long long q = atomicAdd(seq, 1ull) + 1ull;
    reinterpret_cast<volatile unsigned long long*>(host)[2] = q;
    __threadfence_system();
  }
}

// ---- CIC helpers ------------------------------------------------------------------

// Lower tent node and weight of the upper node along one axis for a particle in cell c
// with offset t from the cell's lower face (t may leave [0,1) for X_dagger).
template <typename T>
__device__ __forceinline__ void tent_axis(int c, T t, int n, int& i0, T& f) {
  const T s = t - (T)0.5;
  const T fl = floor(s);
  int i = c + (int)fl;
  T fr = s - fl;
  if (n == 1) { i0 = 0; f = (T)0; return; }
  if (i < 0) { i = 0; fr = (T)0; }
  if (i > n - 2) { i = n - 2; fr = (T)1; }
  i0 = i;
  f = fr;
}

template <typename T>
__device__ __forceinline__ void cic_add(T* grid, const StepConst& K, int i0, int j0, int k0, T fx,
                                        T fy, T fz, T q) {
  const int nx = K.nx, ny = K.ny, nz = K.nz;
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int di = cc & 1, dj = (cc >> 1) & 1, dk = (cc >> 2) & 1;
    const T wt = (di ? fx : (T)1 - fx) * (dj ? fy : (T)1 - fy) * (dk ? fz : (T)1 - fz);
    const int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
    if (wt == (T)0 || ii >= nx || jj >= ny || kk >= nz) continue;
    atomicAdd(&grid[(size_t)ii + (size_t)nx * ((size_t)jj + (size_t)ny * kk)], q * wt);
  }
}

// The field at a particle (CIC interpolation, section "Charge deposition &
// interpolation") from the packed (Ex, Ey, Ez, 0) array: the eight nodes' vectors are
// loaded together (node indices clamped into the grid; a node outside it has weight
// zero and is skipped), then each component is summed in node order.
// The eight node values of a CIC gather (loads only; the weights and the masks of nodes
// outside the grid or of zero weight), then their weighted sums in node order.
template <typename T>
struct CicNodes {
  V4<T> v[8];
  T wt[8];
  bool use[8];
};
template <typename T>
__device__ __forceinline__ void cic_load(const T* E4, const StepConst& K, int i0, int j0, int k0, T fx, T fy,
                                         T fz, CicNodes<T>& g) {
  const int nx = K.nx, ny = K.ny, nz = K.nz;
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int di = cc & 1, dj = (cc >> 1) & 1, dk = (cc >> 2) & 1;
    g.wt[cc] = (di ? fx : (T)1 - fx) * (dj ? fy : (T)1 - fy) * (dk ? fz : (T)1 - fz);
    const int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
    g.use[cc] = !(g.wt[cc] == (T)0 || ii >= nx || jj >= ny || kk >= nz);
    const int ic = ii < nx ? ii : nx - 1, jc = jj < ny ? jj : ny - 1, kc = kk < nz ? kk : nz - 1;
    g.v[cc] = ld4(E4 + 4 * ((size_t)ic + (size_t)nx * ((size_t)jc + (size_t)ny * kc)));
  }
}
template <typename T>
__device__ __forceinline__ void cic_sum(const CicNodes<T>& g, T out[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    T acc = (T)0;
#pragma unroll
    for (int cc = 0; cc < 8; ++cc) acc = g.use[cc] ? acc + g.v[cc].a[a] * g.wt[cc] : acc;
    out[a] = acc;
  }
}
template <typename T>
__device__ __forceinline__ void cic_get3(const T* E4, const StepConst& K, int i0, int j0, int k0, T fx,
                                         T fy, T fz, T out[3]) {
  CicNodes<T> g;
  cic_load<T>(E4, K, i0, j0, k0, fx, fy, fz, g);
  cic_sum<T>(g, out);
}

// ---- TSC (quadratic B-spline) helpers ---------------------------------------------

// Along one axis, for a particle in cell c with offset t from the cell's lower face (t
// may leave [0,1) for X_dagger): nearest cell centre j = c + floor(t), d = t - floor(t)
// - 1/2, weights (1/2 - d)^2 / 2, 3/4 - d^2 and (1/2 + d)^2 / 2 on the centres j - 1, j
// and j + 1; a centre outside the grid hands its weight to the wall cell (the index is
// clamped), so the weights stay a convex combination that sums to one.
template <typename T>
struct Tsc {
  int ix[3], iy[3], iz[3];
  T wx[3], wy[3], wz[3];
};
template <typename T>
__device__ __forceinline__ void tsc_axis(int c, T t, int n, int idx[3], T w[3]) {
  const T fl = floor(t);
  const T d = t - fl - (T)0.5;
  const T lo = (T)0.5 - d, hi = (T)0.5 + d;
  w[0] = (T)0.5 * lo * lo;
  w[1] = (T)0.75 - d * d;
  w[2] = (T)0.5 * hi * hi;
  const int j = c + (int)fl;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int x = j - 1 + q;
    idx[q] = x < 0 ? 0 : (x > n - 1 ? n - 1 : x);
  }
}
template <typename T>
__device__ __forceinline__ Tsc<T> tsc_at(const StepConst& K, int ci, int cj, int ck, T tx, T ty, T tz) {
  Tsc<T> s;
  tsc_axis<T>(ci, tx, K.nx, s.ix, s.wx);
  tsc_axis<T>(cj, ty, K.ny, s.iy, s.wy);
  tsc_axis<T>(ck, tz, K.nz, s.iz, s.wz);
  return s;
}
// The field at a particle from the packed (Ex, Ey, Ez, 0) array: one z plane's nine
// node vectors loaded together, then each component summed in node order (z, y, x),
// weight (wx wy) wz, nodes of zero weight skipped.
template <typename T>
__device__ __forceinline__ void tsc_get3(const T* E4, const StepConst& K, const Tsc<T>& s, T out[3]) {
  const size_t nx = (size_t)K.nx, ny = (size_t)K.ny;
  T acc[3] = {(T)0, (T)0, (T)0};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    V4<T> v[9];
#pragma unroll
    for (int q = 0; q < 9; ++q)
      v[q] = ld4(E4 + 4 * ((size_t)s.ix[q % 3] + nx * ((size_t)s.iy[q / 3] + ny * (size_t)s.iz[c])));
#pragma unroll
    for (int q = 0; q < 9; ++q) {
      const T wt = (s.wx[q % 3] * s.wy[q / 3]) * s.wz[c];
#pragma unroll
      for (int a = 0; a < 3; ++a) acc[a] = wt != (T)0 ? acc[a] + v[q].a[a] * wt : acc[a];
    }
  }
  out[0] = acc[0];
  out[1] = acc[1];
  out[2] = acc[2];
}

// Ion charge (units of e) that cell (i, j, k) receives with the TSC shape: the ions are
// point charges at their cell centres, so along each axis a cell keeps 3/4 of its own
// and takes 1/8 of each neighbour's, and a wall cell also keeps the 1/8 that would fall
// outside.  Every weight is a multiple of 1/512, so the sum is formed in integers: per
// axis the weights in eighths (the cell 6, plus 1 for each wall it touches; each
// neighbour 1, or 0 past a wall), summed along x for each of the nine rows and the rows
// then weighted by y and z.  The total is exact (|total| < 2^53) and so is its scaling
// by 2^-9: the same double as the 27-term sum in any order.
__device__ __forceinline__ void tsc_ion_axis(int c, int n, int w[3], int idx[3]) {
  w[0] = c > 0 ? 1 : 0;
  w[1] = 6 + (c == 0 ? 1 : 0) + (c == n - 1 ? 1 : 0);
  w[2] = c < n - 1 ? 1 : 0;
  idx[0] = c > 0 ? c - 1 : c;  // a tap past the wall reads the cell itself, weight 0
  idx[1] = c;
  idx[2] = c < n - 1 ? c + 1 : c;
}
__device__ __forceinline__ double ion_tsc(const uint32_t* np, const uint32_t* nm, int i, int j, int k,
                                          int nx, int ny, int nz) {
  int wx[3], wy[3], wz[3], xi[3], yj[3], zk[3];
  tsc_ion_axis(i, nx, wx, xi);
  tsc_ion_axis(j, ny, wy, yj);
  tsc_ion_axis(k, nz, wz, zk);
  int64_t acc = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const size_t row = (size_t)nx * ((size_t)yj[b] + (size_t)ny * (size_t)zk[c]);
      int64_t r = 0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const size_t q = row + (size_t)xi[a];
        r += (int64_t)wx[a] * ((int64_t)np[q] - (int64_t)nm[q]);
      }
      acc += (int64_t)(wy[b] * wz[c]) * r;
    }
  }
  return (double)acc * 0x1p-9;
}

template <typename T> struct Mob;
template <> struct Mob<double> {
  __device__ static double mu(const Coef& c, double E) {
    const double Ec = E > c.E_floor ? E : c.E_floor;
    return c.mu_a * pow(Ec / c.mu_E0, c.mu_b);
  }
};
template <> struct Mob<float> {
  // mu_a (E / E0)^b with hardware exp2/log2
  __device__ static float mu(const Coef& c, float E) {
    const float Ec = E > (float)c.E_floor ? E : (float)c.E_floor;
    return (float)c.mu_a *
           __builtin_amdgcn_exp2f((float)c.mu_b * __builtin_amdgcn_logf(Ec / (float)c.mu_E0));
  }
};

template <typename T> struct NormalsF;
template <> struct NormalsF<double> {
  __device__ __forceinline__ static void get(uint4 r, double n[3]) {
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
template <> struct NormalsF<float> {
  __device__ __forceinline__ static void get(uint4 r, float n[3]) {
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

// ---- particle passes --------------------------------------------------------------

// Deposit accumulators.  In single precision the node sums are fixed-point integers
// (conductivity weight mu w in units of 2^-32, electron number in units of 2^-28,
// 64-bit), so a sum does not depend on the order of its atomic additions and the field
// of a realization is bit-reproducible.  A contribution is the product of the
// single-precision tent weight and the particle's integer weight (times the mobility
// for the conductivity), formed in double: the integer weight is not rounded to 24
// bits, so a node that receives all of a particle's charge receives it exactly (a
// quasi-neutral plasma of heavy particles would otherwise carry a spurious charge of
// 2^-24 of its density).  Ranges: 2^31 and 2^35 per node.  Double precision sums
// doubles.
template <typename T> struct DepAcc;
template <> struct DepAcc<double> {
  using S = double;
  __device__ static S enc0(double a) { return a; }
  __device__ static S enc1(double a) { return a; }
  __device__ static double dec0(S v) { return v; }
  __device__ static double dec1(S v) { return v; }
};
template <> struct DepAcc<float> {
  using S = unsigned long long;
  __device__ static S enc0(double a) { return (S)rint(a * 0x1p32); }
  __device__ static S enc1(double a) { return (S)rint(a * 0x1p28); }
  __device__ static double dec0(S v) { return (double)v * 0x1p-32; }
  __device__ static double dec1(S v) { return (double)v * 0x1p-28; }
};

// Charge deposit for the field solve.  A workgroup takes a chunk of kDepChunk
// consecutive (cell-sorted, hence spatially compact) particles and accumulates their
// 8-node CIC contributions in an LDS hash table keyed by grid node (linear probing,
// at most kDepProbes probes, then a direct global atomic); the table is flushed with
// one global atomic per touched node and field.  Mode 0 deposits the electron number
// at X^k only (initial field); mode 1 deposits the conductivity weight mu(|E^k|) w at
// X^k and the electron number at X_dagger (the position after the diffusive part of
// the step, with the normals of the push), and keeps each particle's mobility mu^k for
// the push, which then reads it instead of interpolating E^k again.
// A 1024-entry table per 256-particle chunk, one particle per thread (20 KB of LDS):
// small tables raise the number of resident workgroups, a table four times the chunk
// keeps probing short, and with the row-ordered slots a chunk's nodes rarely collide.
constexpr int kDepChunk = 256;
constexpr int kDepProbes = 8;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
template <typename T> struct DepTbl { static constexpr int log2n = 10; };

template <typename T, int L2>
__device__ __forceinline__ void tbl_add(uint32_t* keys, typename DepAcc<T>::S* v0,
                                        typename DepAcc<T>::S* v1, uint32_t node, uint32_t h, double a,
                                        double b, typename DepAcc<T>::S* g0, typename DepAcc<T>::S* g1) {
  using A = DepAcc<T>;
  constexpr uint32_t mask = (1u << L2) - 1u;
  for (int probe = 0; probe < kDepProbes; ++probe) {
    uint32_t k = keys[h];
    if (k == kEmptyKey) {
      const uint32_t prev = atomicCAS(&keys[h], kEmptyKey, node);
      k = prev == kEmptyKey ? node : prev;
    }
    if (k == node) {
      if (a != 0.0) atomicAdd(&v0[h], A::enc0(a));
      if (b != 0.0) atomicAdd(&v1[h], A::enc1(b));
      return;
    }
    h = (h + 1u) & mask;
  }
  if (a != 0.0) atomicAdd(&g0[node], A::enc0(a));
  if (b != 0.0) atomicAdd(&g1[node], A::enc1(b));
}

// tbl_add for one field and an already encoded (fixed-point) value.
template <int F, int L2>
__device__ __forceinline__ void tbl_add_enc(uint32_t* keys, unsigned long long* v,
                                            uint32_t node, uint32_t h, unsigned long long e,
                                            unsigned long long* g) {
  constexpr uint32_t mask = (1u << L2) - 1u;
  for (int probe = 0; probe < kDepProbes; ++probe) {
    uint32_t k = keys[h];
    if (k == kEmptyKey) {
      const uint32_t prev = atomicCAS(&keys[h], kEmptyKey, node);
      k = prev == kEmptyKey ? node : prev;
    }
    if (k == node) {
      atomicAdd(&v[h], e);
      return;
    }
    h = (h + 1u) & mask;
  }
  atomicAdd(&g[node], e);
}

template <typename T, int L2>
__device__ __forceinline__ void tbl_cic(uint32_t* keys, typename DepAcc<T>::S* v0,
                                        typename DepAcc<T>::S* v1, const StepConst& K, int i0,
                                        int j0, int k0, T fx, T fy, T fz, double qa, double qb,
                                        typename DepAcc<T>::S* g0, typename DepAcc<T>::S* g1) {
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int di = cc & 1, dj = (cc >> 1) & 1, dk = (cc >> 2) & 1;
    const T wt = (di ? fx : (T)1 - fx) * (dj ? fy : (T)1 - fy) * (dk ? fz : (T)1 - fz);
    const int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
    if (wt == (T)0 || ii >= K.nx || jj >= K.ny || kk >= K.nz) continue;
    const uint32_t row = (uint32_t)jj + (uint32_t)K.ny * (uint32_t)kk;
    const uint32_t node = (uint32_t)ii + (uint32_t)K.nx * row;
    // table slot: the row hashed, x kept in order, so that a row's nodes sit in
    // consecutive slots and the flush's atomics of neighbouring lanes share lines
    const uint32_t h = ((uint32_t)ii + ((row * 2654435761u) >> (32 - L2))) & ((1u << L2) - 1u);
    tbl_add<T, L2>(keys, v0, v1, node, h, qa * (double)wt, qb * (double)wt, g0, g1);
  }
}

// The 27 TSC contributions of one particle into the table (clamped wall nodes repeat
// and simply add), with the same slot rule.
template <typename T, int L2>
__device__ __forceinline__ void tbl_tsc(uint32_t* keys, typename DepAcc<T>::S* v0,
                                        typename DepAcc<T>::S* v1, const StepConst& K, const Tsc<T>& s,
                                        double qa, double qb, typename DepAcc<T>::S* g0,
                                        typename DepAcc<T>::S* g1) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const uint32_t row = (uint32_t)s.iy[b] + (uint32_t)K.ny * (uint32_t)s.iz[c];
      const uint32_t hr = (row * 2654435761u) >> (32 - L2);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const T wt = (s.wx[a] * s.wy[b]) * s.wz[c];
        if (wt == (T)0) continue;
        const uint32_t node = (uint32_t)s.ix[a] + (uint32_t)K.nx * row;
        const uint32_t h = ((uint32_t)s.ix[a] + hr) & ((1u << L2) - 1u);
        tbl_add<T, L2>(keys, v0, v1, node, h, qa * (double)wt, qb * (double)wt, g0, g1);
      }
    }
  }
}

// Single precision, TSC shape, one particle per lane (all lanes present; inactive lanes
// contribute nothing).  The lanes of a wavefront hold consecutive, cell-sorted
// particles, and the 27 nodes of a particle depend only on its cell indices j (before
// wall clamping) along the three axes, so the lanes of a run of equal j share them.
// Each node's fixed-point contributions (exact integers: their sum does not depend on
// the order) are summed over every run with a segmented scan, and only the run's last
// lane inserts the sum: a third of the table atomics when cells hold three particles.
// F: 0 conductivity (enc0, v0/g0), 1 electron number (enc1, v1/g1).
template <int F, int L2>
__device__ __forceinline__ void tbl_tsc_runs(uint32_t* keys, unsigned long long* v0,
                                             unsigned long long* v1, const StepConst& K,
                                             const Tsc<float>& s, bool active, int jx, int jy,
                                             int jz, double q, unsigned long long* g0,
                                             unsigned long long* g1) {
  using A = DepAcc<float>;
  const int lane = lane_id();
  // run key: the three cell indices, each biased into 21 bits (an index off the grid by
  // up to 2^20 cells still has a key of its own); inactive lanes all differ from it
  const uint64_t key = active ? ((uint64_t)(uint32_t)(jx + (1 << 20)) << 42) |
                                    ((uint64_t)(uint32_t)(jy + (1 << 20)) << 21) |
                                    (uint64_t)(uint32_t)(jz + (1 << 20))
                              : ~0ull;
  const uint32_t klo = (uint32_t)key, khi = (uint32_t)(key >> 32);
  const uint32_t plo = dpp_from_prev(klo, ~klo), phi = dpp_from_prev(khi, ~khi);
  const uint32_t nlo = dpp_from_next(klo, ~klo), nhi = dpp_from_next(khi, ~khi);
  const uint32_t head = (plo != klo || phi != khi) ? 1u : 0u;
  const bool tail = active && (lane == 63 || nlo != klo || nhi != khi);
  // no run of two or more in the wavefront (sparse cells): every lane inserts its own
  // contributions, as without the run sums, and the scans are skipped
  const bool runs = __ballot(active && lane > 0 && head == 0u) != 0ull;
  const uint64_t zid[1] = {0ull};
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      const uint32_t row = (uint32_t)s.iy[b] + (uint32_t)K.ny * (uint32_t)s.iz[c];
      const uint32_t hr = (row * 2654435761u) >> (32 - L2);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float wt = (s.wx[a] * s.wy[b]) * s.wz[c];
        const double x = q * (double)wt;
        uint64_t v[1] = {active && x != 0.0 ? (F == 0 ? A::enc0(x) : A::enc1(x)) : 0ull};
        if (runs) (void)seg_scan(v, head, zid, [](int, uint64_t u, uint64_t w) { return u + w; });
        if (tail && v[0] != 0ull) {
          const uint32_t node = (uint32_t)s.ix[a] + (uint32_t)K.nx * row;
          const uint32_t h = ((uint32_t)s.ix[a] + hr) & ((1u << L2) - 1u);
          tbl_add_enc<F, L2>(keys, F == 0 ? v0 : v1, node, h, v[0], F == 0 ? g0 : g1);
        }
      }
    }
  }
}

// Single precision: at least 7 waves per SIMD (72 VGPRs, no spills), which measured about
// 3% faster than the compiler's 75 VGPRs and 6 waves in a side-by-side run on the same
// state; 8 waves spill and are slower.  Double precision keeps the compiler's choice (a
// 72-VGPR bound spills).
// The TSC form (SH = 1: 27 nodes per deposit and gather) keeps the compiler's choice.
template <typename T> constexpr int kDepMinWaves = sizeof(T) == 4 ? 7 : 1;
template <typename T, int L2, int SH>
__global__ void __launch_bounds__(256, SH == 0 ? kDepMinWaves<T> : 1) k_field_deposit_lds(Bank a, const Counters* ctr, int which,
                                                          StepConst K, const void* E4, Coef co,
                                                          int mode, typename DepAcc<T>::S* sig,
                                                          typename DepAcc<T>::S* ne, uint32_t chunk,
                                                          T* mu_out) {
  using S = typename DepAcc<T>::S;
  constexpr int TBL = 1 << L2;
  extern __shared__ __align__(16) char smem[];
  S* v0 = reinterpret_cast<S*>(smem);
  S* v1 = v0 + TBL;
  uint32_t* keys = reinterpret_cast<uint32_t*>(v1 + TBL);
  const uint32_t n = min(ctr->n[which], K.cap);
  const T diff = (T)K.diff;
  for (uint32_t c0 = blockIdx.x * chunk; c0 < n; c0 += gridDim.x * chunk) {
    for (int t = threadIdx.x; t < TBL; t += blockDim.x) {
      keys[t] = kEmptyKey;
      v0[t] = (S)0;
      v1[t] = (S)0;
    }
    __syncthreads();
    const uint32_t c1 = min(c0 + chunk, n);
    for (uint32_t ib = c0; ib < c1; ib += blockDim.x) {  // the same trip count in every thread
      const uint32_t i = ib + threadIdx.x;
      const uint32_t w = i < c1 ? a.w[i] : 0u;
      if constexpr (SH == 1 && sizeof(T) == 4) {
        // every lane takes part in the run sums (inactive: weight 0)
        const bool act = w != 0u;
        Tsc<T> sk{}, sd{};
        int jk[3] = {0, 0, 0}, jd[3] = {0, 0, 0};
        double qa = 0.0;
        if (act) {
          const uint32_t cell = a.cell[i];
          int ci, cj, ck;
          cell_ijk(cell, K, ci, cj, ck);
          const T o[3] = {tp<T>(a.ox)[i], tp<T>(a.oy)[i], tp<T>(a.oz)[i]};
          sk = tsc_at<T>(K, ci, cj, ck, o[0], o[1], o[2]);
          jk[0] = ci; jk[1] = cj; jk[2] = ck;
          if (mode != 0) {
            T e[3];
            tsc_get3<T>(ctp<T>(E4), K, sk, e);
            const T Em = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
            const T mu = Mob<T>::mu(co, Em);
            mu_out[i] = mu;
            qa = (double)mu * (double)w;
            const uint64_t id = a.id[i];
            const uint4 r = philox_block((uint32_t)id, (uint32_t)(id >> 32), K.step, TAG_PUSH, 0, K.key);
            T nr[3];
            NormalsF<T>::get(r, nr);
            const T t[3] = {o[0] + diff * nr[0], o[1] + diff * nr[1], o[2] + diff * nr[2]};
            sd = tsc_at<T>(K, ci, cj, ck, t[0], t[1], t[2]);
            jd[0] = ci + (int)floor(t[0]); jd[1] = cj + (int)floor(t[1]); jd[2] = ck + (int)floor(t[2]);
          }
        }
        if (mode == 0) {
          tbl_tsc_runs<1, L2>(keys, v0, v1, K, sk, act, jk[0], jk[1], jk[2], (double)w, sig, ne);
        } else {
          tbl_tsc_runs<0, L2>(keys, v0, v1, K, sk, act, jk[0], jk[1], jk[2], qa, sig, ne);
          tbl_tsc_runs<1, L2>(keys, v0, v1, K, sd, act, jd[0], jd[1], jd[2], (double)w, sig, ne);
        }
        continue;
      }
      if (!w) continue;
      const uint32_t cell = a.cell[i];
      int ci, cj, ck;
      cell_ijk(cell, K, ci, cj, ck);
      const T o[3] = {tp<T>(a.ox)[i], tp<T>(a.oy)[i], tp<T>(a.oz)[i]};
      if constexpr (SH == 0) {
        int i0, j0, k0;
        T fx, fy, fz;
        tent_axis<T>(ci, o[0], K.nx, i0, fx);
        tent_axis<T>(cj, o[1], K.ny, j0, fy);
        tent_axis<T>(ck, o[2], K.nz, k0, fz);
        if (mode == 0) {
          tbl_cic<T, L2>(keys, v0, v1, K, i0, j0, k0, fx, fy, fz, 0.0, (double)w, sig, ne);
          continue;
        }
        T e[3];
        cic_get3<T>(ctp<T>(E4), K, i0, j0, k0, fx, fy, fz, e);
        const T Em = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        const T mu = Mob<T>::mu(co, Em);
        mu_out[i] = mu;
        tbl_cic<T, L2>(keys, v0, v1, K, i0, j0, k0, fx, fy, fz, (double)mu * (double)w, 0.0, sig, ne);
        const uint64_t id = a.id[i];
        const uint4 r = philox_block((uint32_t)id, (uint32_t)(id >> 32), K.step, TAG_PUSH, 0, K.key);
        T nr[3];
        NormalsF<T>::get(r, nr);
        tent_axis<T>(ci, o[0] + diff * nr[0], K.nx, i0, fx);
        tent_axis<T>(cj, o[1] + diff * nr[1], K.ny, j0, fy);
        tent_axis<T>(ck, o[2] + diff * nr[2], K.nz, k0, fz);
        tbl_cic<T, L2>(keys, v0, v1, K, i0, j0, k0, fx, fy, fz, 0.0, (double)w, sig, ne);
      } else {
        const Tsc<T> sk = tsc_at<T>(K, ci, cj, ck, o[0], o[1], o[2]);
        if (mode == 0) {
          tbl_tsc<T, L2>(keys, v0, v1, K, sk, 0.0, (double)w, sig, ne);
          continue;
        }
        T e[3];
        tsc_get3<T>(ctp<T>(E4), K, sk, e);
        const T Em = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
        const T mu = Mob<T>::mu(co, Em);
        mu_out[i] = mu;
        tbl_tsc<T, L2>(keys, v0, v1, K, sk, (double)mu * (double)w, 0.0, sig, ne);
        const uint64_t id = a.id[i];
        const uint4 r = philox_block((uint32_t)id, (uint32_t)(id >> 32), K.step, TAG_PUSH, 0, K.key);
        T nr[3];
        NormalsF<T>::get(r, nr);
        const Tsc<T> sd = tsc_at<T>(K, ci, cj, ck, o[0] + diff * nr[0], o[1] + diff * nr[1], o[2] + diff * nr[2]);
        tbl_tsc<T, L2>(keys, v0, v1, K, sd, 0.0, (double)w, sig, ne);
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < TBL; t += blockDim.x) {
      const uint32_t k = keys[t];
      if (k == kEmptyKey) continue;
      if (v0[t] != (S)0) atomicAdd(&sig[k], v0[t]);
      if (v1[t] != (S)0) atomicAdd(&ne[k], v1[t]);
    }
    __syncthreads();
  }
}

// Semi-implicit push: X^{k+1} = X^k + sqrt(2 D dt) N - mu(|E^k(X^k)|) E^{k+1}(X^k) dt,
// then binning exactly as the uniform push.
template <typename T, int SH>
__global__ void __launch_bounds__(256) k_push_field(Bank a, Counters* ctr, int which,
                                                   unsigned long long* cellacc, uint32_t* tiles,
                                                   StepConst K, const T* mu_in, const void* En4) {
  const uint32_t n = min(ctr->n[which], K.cap);
  const T diff = (T)K.diff;
  const T dtdx = (T)(K.dt / K.dx);
  uint64_t out_w = 0, pushed = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t key = kInvalidCell, w = 0;
    // the particle's own words are read before its weight is tested (one round trip)
    uint32_t cell0 = 0;
    T o0[3] = {(T)0, (T)0, (T)0};
    uint64_t id0 = 0;
    T mu0 = (T)0;
    if (i < n) {
      w = a.w[i];
      cell0 = a.cell[i];
      o0[0] = tp<T>(a.ox)[i];
      o0[1] = tp<T>(a.oy)[i];
      o0[2] = tp<T>(a.oz)[i];
      id0 = a.id[i];
      mu0 = mu_in[i];
    }
    if (w > 0) {
      ++pushed;
      const uint32_t cell = cell0;
      int ci[3];
      cell_ijk(cell, K, ci[0], ci[1], ci[2]);
      T o[3] = {o0[0], o0[1], o0[2]};
      T en[3];
      if constexpr (SH == 0) {
        int i0, j0, k0;
        T fx, fy, fz;
        tent_axis<T>(ci[0], o[0], K.nx, i0, fx);
        tent_axis<T>(ci[1], o[1], K.ny, j0, fy);
        tent_axis<T>(ci[2], o[2], K.nz, k0, fz);
        CicNodes<T> gn;
        cic_load<T>(ctp<T>(En4), K, i0, j0, k0, fx, fy, fz, gn);
        __builtin_amdgcn_sched_barrier(0);  // the eight gathers in flight together
        cic_sum<T>(gn, en);
      } else {
        tsc_get3<T>(ctp<T>(En4), K, tsc_at<T>(K, ci[0], ci[1], ci[2], o[0], o[1], o[2]), en);
      }
      const T mu = mu0;  // mu(|E^k(X^k)|), kept by this step's deposit
      const uint64_t id = id0;
      const uint4 r = philox_block((uint32_t)id, (uint32_t)(id >> 32), K.step, TAG_PUSH, 0, K.key);
      T nr[3];
      NormalsF<T>::get(r, nr);
      const int lim[3] = {K.nx, K.ny, K.nz};
      bool inside = true;
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        T x = (o[ax] + diff * nr[ax]) + (-mu * en[ax]) * dtdx;
        T f = floor(x);
        x -= f;
        if (x >= (T)1) { x -= (T)1; f += (T)1; }
        o[ax] = x;
        ci[ax] += (int)f;
        inside = inside && ci[ax] >= 0 && ci[ax] < lim[ax];
      }
      if (inside) {
        key = (uint32_t)ci[0] + (uint32_t)K.nx * ((uint32_t)ci[1] + (uint32_t)K.ny * (uint32_t)ci[2]);
        a.cell[i] = key;
        tp<T>(a.ox)[i] = o[0];
        tp<T>(a.oy)[i] = o[1];
        tp<T>(a.oz)[i] = o[2];
      } else {
        out_w += w;
        a.w[i] = 0;
      }
    }
    const uint32_t rank = bin_add(cellacc, key, w);
    mark_tile(tiles, key, (uint64_t)rank << 32);
    if (key != kInvalidCell) a.rank[i] = rank;
  }
  out_w = wave_sum64(out_w);
  pushed = wave_sum64(pushed);
  if (lane_id() == 0) {
    if (out_w) atomicAdd(&ctr->outflow, (unsigned long long)out_w);
    if (pushed) atomicAdd(&ctr->pushed, (unsigned long long)pushed);
  }
}

// ---- grid passes ------------------------------------------------------------------

// Storage positions of a cell and of its face neighbours.  Natural order on every
// level: c = i + nx (j + ny k).  Split red-black order on the finest level (nx even):
// an x row keeps its colour-0 cells ((i + j + k) even) at positions 0 .. nx/2 - 1 and
// its colour-1 cells at nx/2 .. nx - 1, each at i / 2.  Every face neighbour has the
// other colour: at the same half-row position in the four neighbouring rows, and at
// the same or the adjacent position in the cell's own row.  A sweep of one colour
// then reads and writes whole lines of each half-row.
struct NatAt {
  ptrdiff_t c, sy, sz;
  __device__ __forceinline__ size_t operator()(int dx, int dy, int dz) const {
    return (size_t)(c + dx + dy * sy + dz * sz);
  }
};

struct SplitAt {
  ptrdiff_t own, oth, sy, sz;
  int odd;  // i & 1
  __device__ __forceinline__ size_t operator()(int dx, int dy, int dz) const {
    if ((dx | dy | dz) == 0) return (size_t)own;
    return (size_t)(oth + (dx < 0 ? odd - 1 : (dx > 0 ? odd : 0)) + dy * sy + dz * sz);
  }
};

__device__ __forceinline__ NatAt nat_at(int i, int j, int k, int nx, int ny) {
  const ptrdiff_t sy = nx, sz = (ptrdiff_t)nx * ny;
  return NatAt{(ptrdiff_t)i + sy * j + sz * k, sy, sz};
}

__device__ __forceinline__ SplitAt split_at(int i, int j, int k, int nx, int ny) {
  const ptrdiff_t sy = nx, sz = (ptrdiff_t)nx * ny;
  const ptrdiff_t row = sy * j + sz * k;
  const int h = nx >> 1, q = (i + j + k) & 1;
  return SplitAt{row + q * h + (i >> 1), row + (1 - q) * h + (i >> 1), sy, sz, i & 1};
}

template <bool kSplit>
__device__ __forceinline__ size_t pos_of(int i, int j, int k, int nx, int ny) {
  if constexpr (kSplit) return (size_t)split_at(i, j, k, nx, ny).own;
  else return (size_t)nat_at(i, j, k, nx, ny).c;
}

template <typename T>
__global__ void k_zero(T* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = (T)0;
}

// Fine-level coefficient (at its storage position) and right-hand side
// b = dx^2 rho / eps0 (+ the lift of the anode potential on the top layer), both
// scaled by dx^2; accumulates ||b||^2.
template <typename T>
__global__ void __launch_bounds__(256) k_field_prep(StepConst K, const uint32_t* nplus,
                                                   const uint32_t* nminus,
                                                   const typename DepAcc<T>::S* ne,
                                                   const typename DepAcc<T>::S* sig,
                                                   double sig_scale, double V, int split, int tsc,
                                                   T* eps, double* b, double* partial) {
  const uint32_t n = K.ncell;
  const double dV = K.dx * K.dx * K.dx;
  const double qscale = K.dx * K.dx * kE / (kEps0 * dV);
  double acc = 0.0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    double bb = 0.0;
    if (c < n) {
      const double e = 1.0 + sig_scale * DepAcc<T>::dec0(sig[c]);
      const uint32_t row = c / (uint32_t)K.nx, k = row / (uint32_t)K.ny;
      const int i = (int)(c - row * (uint32_t)K.nx), j = (int)(row - k * (uint32_t)K.ny);
      eps[split ? pos_of<true>(i, j, (int)k, K.nx, K.ny) : (size_t)c] = (T)e;
      const double ions = tsc ? ion_tsc(nplus, nminus, i, j, (int)k, K.nx, K.ny, K.nz)
                              : (double)nplus[c] - (double)nminus[c];
      const double rho_units = ions - DepAcc<T>::dec1(ne[c]);
      bb = qscale * rho_units;
      if (k == (uint32_t)K.nz - 1) bb += 2.0 * (double)(T)e * V;
      b[c] = bb;
    }
    acc += bb * bb;
  }
  acc = block_sumd(acc);
  if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <typename T>
__global__ void k_eps_restrict(const T* ef, int fnx, int fny, int fsplit, T* ec, int cnx, int cny, int cnz,
                               int csplit) {
  const uint32_t n = (uint32_t)cnx * cny * cnz;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int i = c % cnx, j = (c / cnx) % cny, k = c / (cnx * cny);
    double s = 0.0;
    for (int d = 0; d < 8; ++d) {
      const int fi = 2 * i + (d & 1), fj = 2 * j + ((d >> 1) & 1), fk = 2 * k + (d >> 2);
      s += (double)ef[fsplit ? pos_of<true>(fi, fj, fk, fnx, fny) : pos_of<false>(fi, fj, fk, fnx, fny)];
    }
    ec[csplit ? pos_of<true>(i, j, k, cnx, cny) : (size_t)c] = (T)(s * 0.125);
  }
}

// Harmonic mean for the smoother: exact in double; fast reciprocal in single precision
// (the smoother only has to reduce the error; the double residual of the refinement
// loop defines the solution).
__device__ __forceinline__ double hmean_s(double a, double b) { return 2.0 * a * b / (a + b); }
__device__ __forceinline__ float hmean_s(float a, float b) {
  return (2.0f * a * b) * __builtin_amdgcn_rcpf(a + b);  // v_rcp_f32 (1 ulp), not a full division
}
// The smoother's cell update (f + offsum) / diag, in every smoother form: a division in
// double, the hardware reciprocal in single precision.
__device__ __forceinline__ double smooth_div(double num, double d) { return num / d; }
__device__ __forceinline__ float smooth_div(float num, float d) { return num * __builtin_amdgcn_rcpf(d); }

// Operator of the scaled system at one cell (homogeneous boundary values): sum over
// faces of beta (u_c - u_nb), beta the harmonic mean of the two cells' coefficients,
// plus 2 eps_c u_c on the Dirichlet z faces; x and y faces are Neumann.  Returned as
// the diagonal and the neighbour sum, from the coefficient at the cell and the
// coefficients and values at its six face neighbours (faces ordered x-, x+, y-, y+,
// z-, z+; in[q] false for a face on the domain boundary, whose values are not used: it
// contributes nothing, or the Dirichlet term).  Every finest- and coarse-level kernel
// forms its rows through op_row (working precision) or op_row_r (double accumulation
// for the residual), so all share one arithmetic order.
template <typename T>
__device__ __forceinline__ void op_row(T ec, const T en[6], const T un[6], const bool in[6], T& diag,
                                       T& offsum) {
  T d = 0, s = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const T b = hmean_s(ec, en[q]);
    d = in[q] ? d + b : (q >= 4 ? d + (T)2 * ec : d);
    s = in[q] ? s + b * un[q] : s;
  }
  diag = d;
  offsum = s;
}

// Residual row: face coefficients computed exactly as the smoother computes them
// (single-precision harmonic means in FP32 mode, exact double in FP64 mode), the
// potential and the accumulation in double.
template <typename T>
__device__ __forceinline__ void op_row_r(T ec, const T en[6], const double un[6], const bool in[6],
                                         double& diag, double& offsum) {
  double d = 0, s = 0;
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const double b = (double)hmean_s(ec, en[q]);
    d = in[q] ? d + b : (q >= 4 ? d + 2.0 * (double)ec : d);
    s = in[q] ? s + b * un[q] : s;
  }
  diag = d;
  offsum = s;
}

__device__ __forceinline__ void faces_in(int i, int j, int k, int nx, int ny, int nz, bool in[6]) {
  in[0] = i > 0; in[1] = i < nx - 1; in[2] = j > 0; in[3] = j < ny - 1; in[4] = k > 0; in[5] = k < nz - 1;
}

// Operator row through value accessors a(dx, dy, dz) of the correction and of the
// coefficient at the neighbour (dx, dy, dz) of cell (i, j, k).  All thirteen values
// are read before any arithmetic (offsets clamped to the cell itself on the domain
// faces), so their loads are in flight together.
template <typename T, typename UA, typename EA>
__device__ __forceinline__ void stencil_acc(UA ua, EA ea, int nx, int ny, int nz, int i, int j, int k,
                                            T& diag, T& offsum) {
  bool in[6];
  faces_in(i, j, k, nx, ny, nz, in);
  const int ox[6] = {in[0] ? -1 : 0, in[1] ? 1 : 0, 0, 0, 0, 0};
  const int oy[6] = {0, 0, in[2] ? -1 : 0, in[3] ? 1 : 0, 0, 0};
  const int oz[6] = {0, 0, 0, 0, in[4] ? -1 : 0, in[5] ? 1 : 0};
  const T ec = ea(0, 0, 0);
  T en[6], un[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    en[q] = ea(ox[q], oy[q], oz[q]);
    un[q] = ua(ox[q], oy[q], oz[q]);
  }
  op_row<T>(ec, en, un, in, diag, offsum);
}

template <typename T, typename AT>
__device__ __forceinline__ void stencil_at(const T* u, const T* eps, AT at, int nx, int ny, int nz, int i,
                                           int j, int k, T& diag, T& offsum) {
  stencil_acc<T>([&](int dx, int dy, int dz) { return u[at(dx, dy, dz)]; },
                 [&](int dx, int dy, int dz) { return eps[at(dx, dy, dz)]; }, nx, ny, nz, i, j, k, diag,
                 offsum);
}

template <typename T>
__device__ __forceinline__ void stencil_s(const T* u, const T* eps, int nx, int ny, int nz, int i, int j,
                                          int k, size_t c, T& diag, T& offsum) {
  const ptrdiff_t sy = (ptrdiff_t)nx, sz = (ptrdiff_t)nx * ny;
  stencil_at<T>(u, eps, NatAt{(ptrdiff_t)c, sy, sz}, nx, ny, nz, i, j, k, diag, offsum);
}

// Residual operator row: the potential in natural order, the coefficient through its
// level's positions `at`.
template <typename T, typename AT>
__device__ __forceinline__ void stencil_r(const double* u, const T* eps, AT at, int nx, int ny, int nz,
                                          int i, int j, int k, size_t c, double& diag, double& offsum) {
  const ptrdiff_t sy = (ptrdiff_t)nx, sz = (ptrdiff_t)nx * ny;
  bool in[6];
  faces_in(i, j, k, nx, ny, nz, in);
  const int ox[6] = {in[0] ? -1 : 0, in[1] ? 1 : 0, 0, 0, 0, 0};
  const int oy[6] = {0, 0, in[2] ? -1 : 0, in[3] ? 1 : 0, 0, 0};
  const int oz[6] = {0, 0, 0, 0, in[4] ? -1 : 0, in[5] ? 1 : 0};
  const T ec = eps[at(0, 0, 0)];
  T en[6];
  double un[6];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    en[q] = eps[at(ox[q], oy[q], oz[q])];
    un[q] = u[(size_t)((ptrdiff_t)c + ox[q] + oy[q] * sy + oz[q] * sz)];
  }
  op_row_r<T>(ec, en, un, in, diag, offsum);
}

// Logical (x, y, z) block of a 3-D grid after the XCD remap.
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
  const uint32_t nb = gridDim.x * gridDim.y * gridDim.z;
  const uint32_t lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const uint32_t l = xcd_block(lin, nb);
  bx = (int)(l % gridDim.x);
  by = (int)((l / gridDim.x) % gridDim.y);
  bz = (int)(l / (gridDim.x * gridDim.y));
}

// Gauss-Seidel update of cell (i, j, k) of a level in natural order.
template <typename T>
__device__ __forceinline__ void smooth_cell(T* u, const T* f, const T* eps, int nx, int ny, int nz, int i,
                                            int j, int k) {
  const size_t c = (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k);
  T d, s;
  stencil_s<T>(u, eps, nx, ny, nz, i, j, k, c, d, s);
  u[c] = smooth_div(f[c] + s, d);
}

// One colour of a red-black Gauss-Seidel sweep in natural order: grid (x: half a row,
// y: j, z: k), every thread updates the one cell of the colour in its pair.  kFine
// marks the finest level's instantiation, so that kernel traces report it apart.
template <typename T, bool kFine>
__global__ void __launch_bounds__(128) k_smooth_rb(T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                                  int color) {
  int bx, j, k;
  xcd_block3(bx, j, k);
  const int i = 2 * (int)(bx * blockDim.x + threadIdx.x) + ((j + k + color) & 1);
  if (i >= nx) return;
  smooth_cell<T>(u, f, eps, nx, ny, nz, i, j, k);
}

// One colour of a red-black sweep on the finest level in split order: grid (x: half a
// row, y: j, z: k); the thread at half-row position m updates cell
// i = 2m + ((j + k + colour) & 1), reading its own coefficient and right-hand side and
// the other colour's values, all as whole lines.  Same arithmetic as k_smooth_rb.
template <typename T>
__global__ void __launch_bounds__(128) k_smooth_split(T* u, const T* f, const T* eps, int nx, int ny,
                                                     int nz, int color) {
  int bx, j, k;
  xcd_block3(bx, j, k);
  const int m = (int)(bx * blockDim.x + threadIdx.x);
  if (m >= (nx >> 1)) return;
  const int i = 2 * m + ((j + k + color) & 1);
  const SplitAt at = split_at(i, j, k, nx, ny);
  T d, s;
  stencil_at<T>(u, eps, at, nx, ny, nz, i, j, k, d, s);
  u[at.own] = smooth_div(f[at.own] + s, d);
}

// r = b - A phi in double with the true boundary values (the lift is in b) over
// 256-cell runs, a block taking every gridDim-th run (after the XCD remap); writes the
// working-precision right-hand side of the correction equation and one partial of
// ||r||^2 per block, summed over its runs in order.
constexpr int kResBlocks = 8192;

template <typename T, bool kSplit>
__global__ void __launch_bounds__(256) k_residual_rows(const double* phi, const double* b, const T* eps,
                                                      int nx, int ny, int nz, T* f0, double* partial) {
  const uint32_t n = (uint32_t)nx * ny * nz;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t runs = (n + 255u) / 256u;
  double acc = 0.0;
  for (uint32_t run = blk; run < runs; run += gridDim.x) {
    const uint32_t c = run * 256u + threadIdx.x;
    double rr = 0.0;
    if (c < n) {
      const int i = (int)(c % (uint32_t)nx), j = (int)((c / (uint32_t)nx) % (uint32_t)ny),
                k = (int)(c / ((uint32_t)nx * (uint32_t)ny));
      double d, s;
      size_t q;
      if constexpr (kSplit) {
        const SplitAt at = split_at(i, j, k, nx, ny);
        stencil_r<T>(phi, eps, at, nx, ny, nz, i, j, k, c, d, s);
        q = (size_t)at.own;
      } else {
        const NatAt at = nat_at(i, j, k, nx, ny);
        stencil_r<T>(phi, eps, at, nx, ny, nz, i, j, k, c, d, s);
        q = c;
      }
      rr = b[c] - (d * phi[c] - s);
      f0[q] = (T)rr;
    }
    acc += block_sumd(rr * rr);
  }
  if (threadIdx.x == 0) partial[blk] = acc;
}

// Coarse right-hand side at coarse cell (ci, cj, ck): the sum of its 8 child residuals
// / 2, in the children's order (x offset, then y, then z); zero coarse correction.  The
// fine level in split order if kSplit.
template <typename T, bool kSplit>
__device__ __forceinline__ void restrict_cell(const T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                              T* fc, T* uc, int cnx, int cny, int ci, int cj, int ck) {
  T s8 = 0;
#pragma unroll
  for (int d = 0; d < 8; ++d) {
    const int i = 2 * ci + (d & 1), j = 2 * cj + ((d >> 1) & 1), k = 2 * ck + (d >> 2);
    T dg, sm;
    size_t q;
    if constexpr (kSplit) {
      const SplitAt at = split_at(i, j, k, nx, ny);
      stencil_at<T>(u, eps, at, nx, ny, nz, i, j, k, dg, sm);
      q = (size_t)at.own;
    } else {
      const NatAt at = nat_at(i, j, k, nx, ny);
      stencil_at<T>(u, eps, at, nx, ny, nz, i, j, k, dg, sm);
      q = (size_t)at.c;
    }
    s8 += f[q] - (dg * u[q] - sm);
  }
  const size_t cc = (size_t)ci + (size_t)cnx * ((size_t)cj + (size_t)cny * ck);
  fc[cc] = s8 * (T)0.5;
  uc[cc] = (T)0;
}

// Restriction launch: grid (x: coarse row, y: cj, z: ck).
template <typename T, bool kSplit>
__global__ void __launch_bounds__(128) k_restrict3(const T* u, const T* f, const T* eps, int nx, int ny,
                                                  int nz, T* fc, T* uc, int cnx, int cny) {
  int bx, cj, ck;
  xcd_block3(bx, cj, ck);
  const int ci = bx * blockDim.x + threadIdx.x;
  if (ci >= cnx) return;
  restrict_cell<T, kSplit>(u, f, eps, nx, ny, nz, fc, uc, cnx, cny, ci, cj, ck);
}

// Trilinear prolongation of the coarse correction onto cell centres: along each axis
// the nearer coarse centre weighs 3/4 and the farther 1/4; coarse ghost values mirror
// the cell on the Neumann x and y faces and negate it on the homogeneous Dirichlet z
// faces.  (Second-order transfer: with cell-averaged restriction the transfer orders
// then exceed the order of the operator.)
template <typename T>
__device__ __forceinline__ T prolong_value(const T* uc, int cnx, int cny, int cnz, int i, int j, int k) {
  const int I = i >> 1, J = j >> 1, K = k >> 1;
  const int ia[2] = {I, (i & 1) ? I + 1 : I - 1};
  const int ja[2] = {J, (j & 1) ? J + 1 : J - 1};
  const int ka[2] = {K, (k & 1) ? K + 1 : K - 1};
  const T wt[2] = {(T)0.75, (T)0.25};
  T acc = 0;
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    int a = ia[c & 1], b = ja[(c >> 1) & 1], z = ka[c >> 2];
    a = a < 0 ? 0 : (a >= cnx ? cnx - 1 : a);
    b = b < 0 ? 0 : (b >= cny ? cny - 1 : b);
    T sg = (T)1;
    if (z < 0) { z = 0; sg = (T)-1; }
    if (z >= cnz) { z = cnz - 1; sg = (T)-1; }
    acc += wt[c & 1] * wt[(c >> 1) & 1] * wt[c >> 2] * sg *
           uc[(size_t)a + (size_t)cnx * ((size_t)b + (size_t)cny * z)];
  }
  return acc;
}

template <typename T, bool kSplit>
__global__ void __launch_bounds__(128) k_prolong3(T* u, int nx, int ny, int nz, const T* uc, int cnx,
                                                 int cny, int cnz) {
  int bx, j, k;
  xcd_block3(bx, j, k);
  const int p = bx * blockDim.x + threadIdx.x;  // storage position in the row
  if (p >= nx) return;
  int i = p;
  if constexpr (kSplit) {
    const int h = nx >> 1, q = p >= h ? 1 : 0;
    i = 2 * (p - q * h) + ((j + k + q) & 1);
  }
  u[(size_t)p + (size_t)nx * ((size_t)j + (size_t)ny * k)] += prolong_value<T>(uc, cnx, cny, cnz, i, j, k);
}

// `sweeps` red-black sweeps of a small level inside one workgroup (a barrier between
// colours), the cell updates of the one-colour launches.
template <typename T>
__device__ __forceinline__ void rb_sweeps(T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                          int sweeps) {
  const int n = nx * ny * nz;
  for (int s = 0; s < sweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        if (((i + j + k) & 1) != color) continue;
        smooth_cell<T>(u, f, eps, nx, ny, nz, i, j, k);
      }
      __syncthreads();
    }
}

// Levels of at most kSmallLevel cells: all pre- or post-sweeps in one launch.
constexpr uint32_t kSmallLevel = 4096;
// LDS that one small-level launch may stage: correction, right-hand side and
// coefficient of the level (3 n values).
constexpr size_t kSmallLds = 65536;
template <typename T>
inline bool small_fits_lds(uint32_t n) { return 3 * (size_t)n * sizeof(T) <= kSmallLds; }

template <typename T>
__global__ void __launch_bounds__(1024) k_sweeps_small(T* u, const T* f, const T* eps, int nx, int ny,
                                                      int nz, int sweeps) {
  rb_sweeps<T>(u, f, eps, nx, ny, nz, sweeps);
}

// Launch shapes of the LDS form, threads x cells per thread: levels of up to 64 cells
// run in one wavefront (its barriers cost little), larger ones in 1024 threads x 4
// cells (single precision) or 512 x 8 (double precision, which keeps the registers of
// a thread's cells within its waves' budget).
template <typename T> constexpr int kSmallThreads = sizeof(T) == 8 ? 512 : 1024;
template <typename T> constexpr int kSmallCells = (int)kSmallLevel / kSmallThreads<T>;

// Red-black sweeps of a small level held in LDS, single precision: each of the NT
// threads owns the cells t + r NT (r < NC) and keeps their face coefficients, diagonal
// and right-hand side in registers, so that a sweep reads only the six neighbour
// values.  The coefficients and the update are those of op_row and smooth_cell, in the
// same order (same values).
template <typename T, int NT, int NC>
__device__ __forceinline__ void small_sweeps_cached(T* su, const T* sf, const T* se, int nx, int ny, int nz,
                                                    int sweeps) {
  const int n = nx * ny * nz, sy = nx, sz = nx * ny;
  T bq[NC][6], dg[NC], fr[NC];
  int cr[NC];
  uint32_t meta[NC];  // bits 0-5: face q inside; bit 6: colour; bit 7: owned cell
#pragma unroll
  for (int r = 0; r < NC; ++r) {
    const int c = (int)threadIdx.x + r * NT;
    cr[r] = c < n ? c : 0;
    meta[r] = 0;
    dg[r] = (T)1;
    fr[r] = (T)0;
    if (c < n) {
      const int i = c % nx, j = (c / nx) % ny, k = c / sz;
      bool in[6];
      faces_in(i, j, k, nx, ny, nz, in);
      const int off[6] = {in[0] ? -1 : 0, in[1] ? 1 : 0, in[2] ? -sy : 0,
                          in[3] ? sy : 0, in[4] ? -sz : 0, in[5] ? sz : 0};
      const T ec = se[c];
      T d = 0;
      uint32_t m = 0x80u | ((uint32_t)((i + j + k) & 1) << 6);
#pragma unroll
      for (int q = 0; q < 6; ++q) {
        const T b = hmean_s(ec, se[c + off[q]]);
        bq[r][q] = b;
        d = in[q] ? d + b : (q >= 4 ? d + (T)2 * ec : d);
        m |= in[q] ? (1u << q) : 0u;
      }
      dg[r] = d;
      fr[r] = sf[c];
      meta[r] = m;
    }
  }
  for (int it = 0; it < sweeps; ++it)
    for (int color = 0; color < 2; ++color) {
      const uint32_t want = 0x80u | ((uint32_t)color << 6);
#pragma unroll
      for (int r = 0; r < NC; ++r) {
        if ((meta[r] & 0xC0u) != want) continue;
        const int c = cr[r];
        const uint32_t m = meta[r];
        const int off[6] = {(m & 1u) ? -1 : 0, (m & 2u) ? 1 : 0, (m & 4u) ? -sy : 0,
                            (m & 8u) ? sy : 0, (m & 16u) ? -sz : 0, (m & 32u) ? sz : 0};
        T un[6];
#pragma unroll
        for (int q = 0; q < 6; ++q) un[q] = su[c + off[q]];
        T acc = 0;
#pragma unroll
        for (int q = 0; q < 6; ++q) acc = ((m >> q) & 1u) ? acc + bq[r][q] * un[q] : acc;
        su[c] = smooth_div(fr[r] + acc, dg[r]);
      }
      __syncthreads();
    }
}

// A small level staged in LDS by NT threads, NC cells each (the host checks
// small_fits_lds and n <= NT NC): the level's coefficient and right-hand side and its
// correction (plus the prolonged coarse correction if uc_in, zero if zero_u) are
// loaded once, all loads of a thread in flight together; every sweep runs on the LDS
// copies with the cell updates of the one-colour launches (same values), and the
// correction is stored back; with fc_out the level's residual is then restricted to
// the next coarser level (its correction zeroed), as the restriction launch does.
template <typename T, int NT, int NC>
__global__ void __launch_bounds__(NT) k_small_lds(T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                                 int sweeps, bool zero_u, const T* uc_in, T* fc_out,
                                                 T* uc_out, int cnx, int cny, int cnz) {
  extern __shared__ __align__(16) char smem[];
  const int n = nx * ny * nz;
  T* su = reinterpret_cast<T*>(smem);
  T* sf = su + n;
  T* se = sf + n;
  T vu[NC], vf[NC], ve[NC];
#pragma unroll
  for (int r = 0; r < NC; ++r) {
    const int c = (int)threadIdx.x + r * NT;
    vu[r] = vf[r] = ve[r] = (T)0;
    if (c < n) {
      vu[r] = zero_u ? (T)0 : u[c];
      vf[r] = f[c];
      ve[r] = eps[c];
    }
  }
  if (uc_in) {
#pragma unroll
    for (int r = 0; r < NC; ++r) {
      const int c = (int)threadIdx.x + r * NT;
      if (c < n) {
        const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        vu[r] = vu[r] + prolong_value<T>(uc_in, cnx, cny, cnz, i, j, k);
      }
    }
  }
#pragma unroll
  for (int r = 0; r < NC; ++r) {
    const int c = (int)threadIdx.x + r * NT;
    if (c < n) {
      su[c] = vu[r];
      sf[c] = vf[r];
      se[c] = ve[r];
    }
  }
  __syncthreads();
  if constexpr (sizeof(T) == 4)
    small_sweeps_cached<T, NT, NC>(su, sf, se, nx, ny, nz, sweeps);
  else
    rb_sweeps<T>(su, sf, se, nx, ny, nz, sweeps);
#pragma unroll
  for (int r = 0; r < NC; ++r) {
    const int c = (int)threadIdx.x + r * NT;
    if (c < n) u[c] = su[c];
  }
  if (fc_out) {
    const int cn = cnx * cny * cnz;
    for (int q = threadIdx.x; q < cn; q += NT) {
      const int ci = q % cnx, cj = (q / cnx) % cny, ck = q / (cnx * cny);
      restrict_cell<T, false>(su, sf, se, nx, ny, nz, fc_out, uc_out, cnx, cny, ci, cj, ck);
    }
  }
}

// Launch of the LDS form on a level of n cells (n <= kSmallLevel, small_fits_lds).
template <typename T>
static void launch_small_lds(hipStream_t s, uint32_t n, T* u, const T* f, const T* eps, int nx, int ny,
                             int nz, int sweeps, bool zero_u, const T* uc_in, T* fc_out, T* uc_out, int cnx,
                             int cny, int cnz) {
  const size_t lds = 3 * (size_t)n * sizeof(T);
  if (n <= 64)
    k_small_lds<T, 64, 1><<<1, 64, lds, s>>>(u, f, eps, nx, ny, nz, sweeps, zero_u, uc_in, fc_out, uc_out,
                                             cnx, cny, cnz);
  else
    k_small_lds<T, kSmallThreads<T>, kSmallCells<T>><<<1, kSmallThreads<T>, lds, s>>>(
        u, f, eps, nx, ny, nz, sweeps, zero_u, uc_in, fc_out, uc_out, cnx, cny, cnz);
}

// Coarsest level: red-black sweeps from zero inside one workgroup (levels too large
// for the LDS form).
template <typename T>
__global__ void __launch_bounds__(1024) k_bottom(T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                                int sweeps) {
  const int n = nx * ny * nz;
  for (int c = threadIdx.x; c < n; c += blockDim.x) u[c] = (T)0;
  __syncthreads();
  rb_sweeps<T>(u, f, eps, nx, ny, nz, sweeps);
}

// ---- finest level over row segments ---------------------------------------------------
// With nx a multiple of 8 the finest-level kernels give each thread a segment of eight
// cells of an x row (i = 8t .. 8t+7; the smoother: four cells of one colour).  In split
// order a segment is positions 4t .. 4t+3 of both half rows, in natural order eight
// consecutive values, so every access to the level's arrays is a 16-byte vector.  The
// per-cell arithmetic is op_row / op_row_r, as in the one-cell kernels, and both orders
// run the same segment kernels (the smoother has no reduction and is order-free), so
// their results are identical.

// Cells 8t .. 8t+7 of the finest-level row starting at rb (parity par = (j + k) & 1),
// in natural order; h = nx / 2.  Cell 8t + 2r + e has colour (e + par) & 1 and sits at
// position 4t + r of that colour's half row.
template <typename T, bool kSplit>
__device__ __forceinline__ void ld_seg(const T* a, size_t rb, int h, int t, int par, T v[8]) {
  if constexpr (kSplit) {
    const V4<T> c0 = ld4(a + rb + 4 * t), c1 = ld4(a + rb + h + 4 * t);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[2 * r] = par ? c1.a[r] : c0.a[r];
      v[2 * r + 1] = par ? c0.a[r] : c1.a[r];
    }
  } else {
    const V4<T> a0 = ld4(a + rb + 8 * t), a1 = ld4(a + rb + 8 * t + 4);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      v[r] = a0.a[r];
      v[4 + r] = a1.a[r];
    }
  }
}

template <typename T, bool kSplit>
__device__ __forceinline__ void st_seg(T* a, size_t rb, int h, int t, int par, const T v[8]) {
  if constexpr (kSplit) {
    const int e0 = par, e1 = 1 - par;  // the natural parity of the colour-0 and colour-1 cells
    st4<T>(a + rb + 4 * t, v[e0], v[2 + e0], v[4 + e0], v[6 + e0]);
    st4<T>(a + rb + h + 4 * t, v[e1], v[2 + e1], v[4 + e1], v[6 + e1]);
  } else {
    st4<T>(a + rb + 8 * t, v[0], v[1], v[2], v[3]);
    st4<T>(a + rb + 8 * t + 4, v[4], v[5], v[6], v[7]);
  }
}

template <typename T, bool kSplit>
__device__ __forceinline__ T ld_cell(const T* a, size_t rb, int h, int i, int par) {
  if constexpr (kSplit) return a[rb + (((i + par) & 1) ? (size_t)h : 0) + (size_t)(i >> 1)];
  else return a[rb + (size_t)i];
}

// Segment g of a level with ns segments per row: row index, t, j, k, parity.
struct Seg {
  uint32_t row;
  int t, j, k, par;
};

__device__ __forceinline__ Seg seg_of(uint32_t g, int ns, int ny) {
  Seg s;
  s.row = g / (uint32_t)ns;
  s.t = (int)(g - s.row * (uint32_t)ns);
  s.k = (int)(s.row / (uint32_t)ny);
  s.j = (int)(s.row - (uint32_t)s.k * (uint32_t)ny);
  s.par = (s.j + s.k) & 1;
  return s;
}

// The segment's row and its four neighbouring rows (each replaced by the row itself
// where there is none: those values are not used), with their parities.
struct SegRows {
  size_t rb, ym, yp, zm, zp;
  int pym, pyp, pzm, pzp;
};

__device__ __forceinline__ SegRows seg_rows(const Seg& s, int nx, int ny, int nz) {
  SegRows R;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  R.rb = (size_t)s.row * sy;
  R.ym = s.j > 0 ? R.rb - sy : R.rb;
  R.yp = s.j < ny - 1 ? R.rb + sy : R.rb;
  R.zm = s.k > 0 ? R.rb - sz : R.rb;
  R.zp = s.k < nz - 1 ? R.rb + sz : R.rb;
  R.pym = s.j > 0 ? s.par ^ 1 : s.par;
  R.pyp = s.j < ny - 1 ? s.par ^ 1 : s.par;
  R.pzm = s.k > 0 ? s.par ^ 1 : s.par;
  R.pzp = s.k < nz - 1 ? s.par ^ 1 : s.par;
  return R;
}

// A segment's values of one array: the eight cells, the cells before and after it in
// the row (clamped to the segment at the row ends), and the same eight cells of the
// four neighbouring rows.
template <typename T>
struct SegVals {
  T c[8], ym[8], yp[8], zm[8], zp[8];
  T l, r;
};

template <typename T, bool kSplit>
__device__ __forceinline__ void ld_seg_vals(const T* a, const SegRows& R, const Seg& s, int nx, SegVals<T>& v) {
  const int h = nx >> 1, i0 = 8 * s.t;
  ld_seg<T, kSplit>(a, R.rb, h, s.t, s.par, v.c);
  ld_seg<T, kSplit>(a, R.ym, h, s.t, R.pym, v.ym);
  ld_seg<T, kSplit>(a, R.yp, h, s.t, R.pyp, v.yp);
  ld_seg<T, kSplit>(a, R.zm, h, s.t, R.pzm, v.zm);
  ld_seg<T, kSplit>(a, R.zp, h, s.t, R.pzp, v.zp);
  v.l = ld_cell<T, kSplit>(a, R.rb, h, i0 > 0 ? i0 - 1 : i0, s.par);
  v.r = ld_cell<T, kSplit>(a, R.rb, h, i0 + 8 < nx ? i0 + 8 : i0 + 7, s.par);
}

// Face-neighbour values of cell r of the segment (faces ordered as in op_row).
template <typename T>
__device__ __forceinline__ void seg_faces(const SegVals<T>& v, int r, T out[6]) {
  out[0] = r > 0 ? v.c[r - 1] : v.l;
  out[1] = r < 7 ? v.c[r + 1] : v.r;
  out[2] = v.ym[r];
  out[3] = v.yp[r];
  out[4] = v.zm[r];
  out[5] = v.zp[r];
}

// Double residual over segments (as k_residual_rows: a block takes every gridDim-th run
// of 256 segments; one partial of ||r||^2 per block, each thread's eight cells summed
// in order).
template <typename T, bool kSplit>
__global__ void __launch_bounds__(256) k_residual_seg(const double* phi, const double* b, const T* eps,
                                                     int nx, int ny, int nz, T* f0, double* partial) {
  const int ns = nx >> 3, h = nx >> 1;
  const uint32_t nseg = (uint32_t)ns * ny * nz;
  const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
  const uint32_t runs = (nseg + 255u) / 256u;
  double acc = 0.0;
  for (uint32_t run = blk; run < runs; run += gridDim.x) {
    const uint32_t g = run * 256u + threadIdx.x;
    double rs = 0.0;
    if (g < nseg) {
      const Seg s = seg_of(g, ns, ny);
      const SegRows R = seg_rows(s, nx, ny, nz);
      const int i0 = 8 * s.t;
      // two rounds of loads, each issued together before its arithmetic: the segment's
      // row with its x and y neighbours (faces 0-3), then the z neighbour rows (faces
      // 4-5); the face sums continue in the operator's face order (same values), and
      // the y rows are dead before the z rows arrive (fewer registers, more waves)
      double Pc[8], Pym[8], Pyp[8], B[8];
      T Ec[8], Eym[8], Eyp[8];
      ld_seg<double, false>(phi, R.rb, h, s.t, s.par, Pc);
      ld_seg<double, false>(phi, R.ym, h, s.t, R.pym, Pym);
      ld_seg<double, false>(phi, R.yp, h, s.t, R.pyp, Pyp);
      const double Pl = ld_cell<double, false>(phi, R.rb, h, i0 > 0 ? i0 - 1 : i0, s.par);
      const double Pr = ld_cell<double, false>(phi, R.rb, h, i0 + 8 < nx ? i0 + 8 : i0 + 7, s.par);
      ld_seg<T, kSplit>(eps, R.rb, h, s.t, s.par, Ec);
      ld_seg<T, kSplit>(eps, R.ym, h, s.t, R.pym, Eym);
      ld_seg<T, kSplit>(eps, R.yp, h, s.t, R.pyp, Eyp);
      const T El = ld_cell<T, kSplit>(eps, R.rb, h, i0 > 0 ? i0 - 1 : i0, s.par);
      const T Er = ld_cell<T, kSplit>(eps, R.rb, h, i0 + 8 < nx ? i0 + 8 : i0 + 7, s.par);
      ld_seg<double, false>(b, R.rb, h, s.t, s.par, B);
      __builtin_amdgcn_sched_barrier(0);
      double d[8], sm[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        bool in[6];
        faces_in(i0 + r, s.j, s.k, nx, ny, nz, in);
        const T en[4] = {r > 0 ? Ec[r - 1] : El, r < 7 ? Ec[r + 1] : Er, Eym[r], Eyp[r]};
        const double un[4] = {r > 0 ? Pc[r - 1] : Pl, r < 7 ? Pc[r + 1] : Pr, Pym[r], Pyp[r]};
        double dd = 0, ss = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const double bq = (double)hmean_s(Ec[r], en[q]);
          dd = in[q] ? dd + bq : dd;
          ss = in[q] ? ss + bq * un[q] : ss;
        }
        d[r] = dd;
        sm[r] = ss;
      }
      __builtin_amdgcn_sched_barrier(0);  // the z rows are loaded after the y rows are dead
      double Pzm[8], Pzp[8];
      T Ezm[8], Ezp[8];
      ld_seg<double, false>(phi, R.zm, h, s.t, R.pzm, Pzm);
      ld_seg<double, false>(phi, R.zp, h, s.t, R.pzp, Pzp);
      ld_seg<T, kSplit>(eps, R.zm, h, s.t, R.pzm, Ezm);
      ld_seg<T, kSplit>(eps, R.zp, h, s.t, R.pzp, Ezp);
      __builtin_amdgcn_sched_barrier(0);
      T F[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        const bool in4 = s.k > 0, in5 = s.k < nz - 1;
        double dd = d[r], ss = sm[r];
        {
          const double bq = (double)hmean_s(Ec[r], Ezm[r]);
          dd = in4 ? dd + bq : dd + 2.0 * (double)Ec[r];
          ss = in4 ? ss + bq * Pzm[r] : ss;
        }
        {
          const double bq = (double)hmean_s(Ec[r], Ezp[r]);
          dd = in5 ? dd + bq : dd + 2.0 * (double)Ec[r];
          ss = in5 ? ss + bq * Pzp[r] : ss;
        }
        const double rr = B[r] - (dd * Pc[r] - ss);
        F[r] = (T)rr;
        rs += rr * rr;
      }
      st_seg<T, kSplit>(f0, R.rb, h, s.t, s.par, F);
    }
    acc += block_sumd(rs);
  }
  if (threadIdx.x == 0) partial[blk] = acc;
}

// One colour of a red-black sweep on a split segment level, four cells of the colour
// per thread (kFine marks the finest level's instantiation for kernel traces): cells i = 2m + odd for half-row positions m = 4t .. 4t+3, odd =
// (j + k + colour) & 1.  Their x neighbours have the other colour, at positions
// m - 1 + odd and m + odd.
template <typename T, bool kFine, bool kZero = false>
__global__ void __launch_bounds__(256) k_smooth_seg(T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                                   int color) {
  const int ns = nx >> 3, h = nx >> 1;
  const uint32_t g = xcd_block(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (g >= (uint32_t)ns * ny * nz) return;
  const Seg s = seg_of(g, ns, ny);
  const int odd = (s.par + color) & 1;
  const size_t rb = (size_t)s.row * nx;
  const size_t own = rb + (color ? (size_t)h : 0) + 4 * s.t, oth = rb + (color ? 0 : (size_t)h) + 4 * s.t;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  const size_t oym = s.j > 0 ? oth - sy : oth, oyp = s.j < ny - 1 ? oth + sy : oth;
  const size_t ozm = s.k > 0 ? oth - sz : oth, ozp = s.k < nz - 1 ? oth + sz : oth;
  // the one x neighbour outside the segment's other-colour values: on the left of the
  // first cell (odd = 0) or on the right of the last (odd = 1); a single unconditional
  // load, so that it joins the others in flight
  const size_t pe = odd ? (4 * s.t + 4 < h ? oth + 4 : oth + 3) : (s.t > 0 ? oth - 1 : oth);
  const V4<T> Fo = ld4(f + own), Eo = ld4(eps + own);
  const V4<T> Ec = ld4(eps + oth);
  const V4<T> Eym = ld4(eps + oym), Eyp = ld4(eps + oyp), Ezm = ld4(eps + ozm), Ezp = ld4(eps + ozp);
  const T EX = eps[pe];
  // kZero: the first colour-0 sweep of a cycle, from u = 0 (the neighbours' values are
  // zeros, not read)
  const V4<T> zero = {{(T)0, (T)0, (T)0, (T)0}};
  const V4<T> Uc = kZero ? zero : ld4(u + oth);
  const V4<T> Uym = kZero ? zero : ld4(u + oym), Uyp = kZero ? zero : ld4(u + oyp);
  const V4<T> Uzm = kZero ? zero : ld4(u + ozm), Uzp = kZero ? zero : ld4(u + ozp);
  const T UX = kZero ? (T)0 : u[pe];
  __builtin_amdgcn_sched_barrier(0);  // all loads issued before the arithmetic
  T un_[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    bool in[6];
    faces_in(2 * (4 * s.t + r) + odd, s.j, s.k, nx, ny, nz, in);
    const T en[6] = {odd ? Ec.a[r] : (r > 0 ? Ec.a[r - 1] : EX), odd ? (r < 3 ? Ec.a[r + 1] : EX) : Ec.a[r],
                     Eym.a[r], Eyp.a[r], Ezm.a[r], Ezp.a[r]};
    const T un[6] = {odd ? Uc.a[r] : (r > 0 ? Uc.a[r - 1] : UX), odd ? (r < 3 ? Uc.a[r + 1] : UX) : Uc.a[r],
                     Uym.a[r], Uyp.a[r], Uzm.a[r], Uzp.a[r]};
    T d, sm;
    op_row<T>(Eo.a[r], en, un, in, d, sm);
    un_[r] = smooth_div(Fo.a[r] + sm, d);
  }
  st4<T>(u + own, un_[0], un_[1], un_[2], un_[3]);
}

// Restriction from a segment level: a thread takes four coarse cells (coarse x
// 4t .. 4t+3) and their children, the fine segment t of four fine rows, visited in the
// children's order (j offset, then k offset; x offset within a row), so each coarse
// sum adds its eight child residuals in the order of k_restrict3.  The fine level in
// split order if kSplit, the coarse one if kCSplit (coarse cells 4t, 4t+1 sit at
// half-row position 2t, 4t+2 and 4t+3 at 2t+1, one of each pair in each half).
template <typename T, bool kSplit, bool kCSplit>
__global__ void __launch_bounds__(256) k_restrict_seg(const T* u, const T* f, const T* eps, int nx, int ny,
                                                     int nz, T* fc, T* uc) {
  const int ns = nx >> 3, h = nx >> 1, cnx = nx >> 1, cny = ny >> 1, cnz = nz >> 1;
  const uint32_t g = xcd_block(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (g >= (uint32_t)ns * cny * cnz) return;
  const Seg cs = seg_of(g, ns, cny);
  T s8[4] = {0, 0, 0, 0};
#pragma unroll 1
  for (int dd = 0; dd < 4; ++dd) {
    Seg s;
    s.t = cs.t;
    s.j = 2 * cs.j + (dd & 1);
    s.k = 2 * cs.k + (dd >> 1);
    s.row = (uint32_t)s.j + (uint32_t)ny * (uint32_t)s.k;
    s.par = (s.j + s.k) & 1;
    const SegRows R = seg_rows(s, nx, ny, nz);
    SegVals<T> U, E;
    ld_seg_vals<T, kSplit>(u, R, s, nx, U);
    ld_seg_vals<T, kSplit>(eps, R, s, nx, E);
    T F[8];
    ld_seg<T, kSplit>(f, R.rb, h, s.t, s.par, F);
    __builtin_amdgcn_sched_barrier(0);  // the row's loads in flight together
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      bool in[6];
      faces_in(8 * s.t + r, s.j, s.k, nx, ny, nz, in);
      T en[6], un[6];
      seg_faces(E, r, en);
      seg_faces(U, r, un);
      T dg, sm;
      op_row<T>(E.c[r], en, un, in, dg, sm);
      s8[r >> 1] += F[r] - (dg * U.c[r] - sm);
    }
  }
  const size_t cb = (size_t)cs.row * cnx;
  if constexpr (kCSplit) {
    const int ch = cnx >> 1;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int ci = 4 * cs.t + r;
      const size_t q = cb + (((ci + cs.par) & 1) ? (size_t)ch : 0) + (size_t)(ci >> 1);
      fc[q] = s8[r] * (T)0.5;
      uc[q] = (T)0;
    }
  } else {
    st4<T>(fc + cb + 4 * cs.t, s8[0] * (T)0.5, s8[1] * (T)0.5, s8[2] * (T)0.5, s8[3] * (T)0.5);
    st4<T>(uc + cb + 4 * cs.t, (T)0, (T)0, (T)0, (T)0);
  }
}

// Trilinear prolongation onto the finest level over segments: the coarse values of
// the eight cells come from the coarse rows (J or its neighbour toward the cell) x
// (K or its neighbour), x from 4t-1 to 4t+4 with the clamps and Dirichlet signs of
// k_prolong3, in the same order and arithmetic.
template <typename T, bool kSplit, bool kCSplit>
__global__ void __launch_bounds__(256) k_prolong_seg(T* u, int nx, int ny, int nz, const T* uc, int cnx,
                                                    int cny, int cnz) {
  const int ns = nx >> 3, h = nx >> 1;
  const uint32_t g = xcd_block(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (g >= (uint32_t)ns * ny * nz) return;
  const Seg s = seg_of(g, ns, ny);
  const int J = s.j >> 1, K = s.k >> 1;
  const int jb = (s.j & 1) ? J + 1 : J - 1, kb = (s.k & 1) ? K + 1 : K - 1;
  const int jbc = jb < 0 ? 0 : (jb >= cny ? cny - 1 : jb);
  const int kbc = kb < 0 ? 0 : (kb >= cnz ? cnz - 1 : kb);
  const T sgk = (kb < 0 || kb >= cnz) ? (T)-1 : (T)1;
  T W[2][2][6];
#pragma unroll
  for (int dj = 0; dj < 2; ++dj)
#pragma unroll
    for (int dk = 0; dk < 2; ++dk) {
      const int rj = dj ? jbc : J, rk = dk ? kbc : K;
      const size_t crow = (size_t)cnx * ((size_t)rj + (size_t)cny * (size_t)rk);
      const int xl = s.t > 0 ? 4 * s.t - 1 : 0, xr = 4 * s.t + 4 < cnx ? 4 * s.t + 4 : cnx - 1;
      if constexpr (kCSplit) {
        const int ch = cnx >> 1, cp = (rj + rk) & 1;
        auto cv = [&](int x) { return uc[crow + (((x + cp) & 1) ? (size_t)ch : 0) + (size_t)(x >> 1)]; };
        W[dj][dk][0] = cv(xl);
#pragma unroll
        for (int q = 0; q < 4; ++q) W[dj][dk][1 + q] = cv(4 * s.t + q);
        W[dj][dk][5] = cv(xr);
      } else {
        const V4<T> m = ld4(uc + crow + 4 * s.t);
        W[dj][dk][0] = uc[crow + xl];
        W[dj][dk][1] = m.a[0]; W[dj][dk][2] = m.a[1]; W[dj][dk][3] = m.a[2]; W[dj][dk][4] = m.a[3];
        W[dj][dk][5] = uc[crow + xr];
      }
    }
  const size_t rb = (size_t)s.row * nx;
  T V[8];
  ld_seg<T, kSplit>(u, rb, h, s.t, s.par, V);
  const T wt[2] = {(T)0.75, (T)0.25};
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    T acc = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      // x: I = 4t + r/2 sits at window index r/2 + 1; the far neighbour is I + 1 for
      // odd i and I - 1 for even i
      const int xa = (c & 1) ? ((r & 1) ? (r >> 1) + 2 : (r >> 1)) : (r >> 1) + 1;
      const T sg = (c >> 2) ? sgk : (T)1;
      acc += wt[c & 1] * wt[(c >> 1) & 1] * wt[c >> 2] * sg * W[(c >> 1) & 1][c >> 2][xa];
    }
    V[r] += acc;
  }
  st_seg<T, kSplit>(u, rb, h, s.t, s.par, V);
}

// phi += u over the finest level, a segment per thread.
template <typename T, bool kSplit>
__global__ void __launch_bounds__(256) k_phi_update_seg(double* phi, const T* u, int nx, int ny, int nz) {
  const int ns = nx >> 3, h = nx >> 1;
  const uint32_t g = xcd_block(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (g >= (uint32_t)ns * ny * nz) return;
  const Seg s = seg_of(g, ns, ny);
  const size_t rb = (size_t)s.row * nx;
  T V[8];
  double P[8];
  ld_seg<T, kSplit>(u, rb, h, s.t, s.par, V);
  ld_seg<double, false>(phi, rb, h, s.t, s.par, P);
#pragma unroll
  for (int r = 0; r < 8; ++r) P[r] += (double)V[r];
  st_seg<double, false>(phi, rb, h, s.t, s.par, P);
}

// Initial guess by linear extrapolation in time: phi <- 2 phi - prev, prev <- old phi.
__global__ void k_extrapolate(double* phi, double* prev, uint32_t n, int have_prev) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const double p = phi[c];
    if (have_prev) phi[c] = 2.0 * p - prev[c];
    prev[c] = p;
  }
}

// phi += u over the finest level; grid (x: row position, y: j, z: k), u read in its
// storage order.
template <typename T, bool kSplit>
__global__ void __launch_bounds__(128) k_phi_update(double* phi, const T* u, int nx, int ny) {
  int bx, j, k;
  xcd_block3(bx, j, k);
  const int p = bx * blockDim.x + threadIdx.x;
  if (p >= nx) return;
  int i = p;
  if constexpr (kSplit) {
    const int h = nx >> 1, q = p >= h ? 1 : 0;
    i = 2 * (p - q * h) + ((j + k + q) & 1);
  }
  const size_t row = (size_t)nx * ((size_t)j + (size_t)ny * k);
  phi[row + i] += (double)u[row + p];
}

// E = -grad phi at cell centres into the packed (Ex, Ey, Ez, 0) array.
template <typename T>
__global__ void k_efield(const double* phi, int nx, int ny, int nz, double V, double inv2h, T* E4) {
  const uint32_t n = (uint32_t)nx * ny * nz;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    // neighbour indices clamped to the cell itself on the faces, so the seven loads are
    // unconditional and in flight together (the clamped value is the Neumann one)
    const double pc = phi[c];
    const double xm = phi[i > 0 ? c - 1 : c], xp = phi[i < nx - 1 ? c + 1 : c];
    const double ym = phi[j > 0 ? c - sy : c], yp = phi[j < ny - 1 ? c + sy : c];
    const double vzm = phi[k > 0 ? c - sz : c], vzp = phi[k < nz - 1 ? c + sz : c];
    __builtin_amdgcn_sched_barrier(0);
    const double zm = k > 0 ? vzm : -pc, zp = k < nz - 1 ? vzp : 2.0 * V - pc;
    st4<T>(E4 + 4 * (size_t)c, (T)(-(xp - xm) * inv2h), (T)(-(yp - ym) * inv2h), (T)(-(zp - zm) * inv2h),
           (T)0);
  }
}

// The same field over 4-cell row segments (nx a multiple of 4): a thread reads the
// potential of its four cells and of the four cells of each neighbouring row as
// 16-byte vectors, plus the cells before and after the segment, all in flight
// together, and writes four packed values; each cell's differences are those of
// k_efield (same values).
template <typename T>
__global__ void __launch_bounds__(256) k_efield_seg(const double* phi, int nx, int ny, int nz, double V,
                                                   double inv2h, T* E4) {
  const int ns = nx >> 2;
  const uint32_t nseg = (uint32_t)ns * ny * nz;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  for (uint32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < nseg; g += gridDim.x * blockDim.x) {
    const uint32_t row = g / (uint32_t)ns;
    const int t = (int)(g - row * (uint32_t)ns);
    const int j = (int)(row % (uint32_t)ny), k = (int)(row / (uint32_t)ny);
    const size_t c0 = (size_t)row * sy + 4 * (size_t)t;
    const V4<double> pc = ld4(phi + c0);
    const V4<double> ym = ld4(phi + (j > 0 ? c0 - sy : c0)), yp = ld4(phi + (j < ny - 1 ? c0 + sy : c0));
    const V4<double> zm = ld4(phi + (k > 0 ? c0 - sz : c0)), zp = ld4(phi + (k < nz - 1 ? c0 + sz : c0));
    const double pl = phi[t > 0 ? c0 - 1 : c0], pr = phi[4 * t + 4 < nx ? c0 + 4 : c0 + 3];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double xm = r > 0 ? pc.a[r - 1] : pl, xp = r < 3 ? pc.a[r + 1] : pr;
      const double vzm = k > 0 ? zm.a[r] : -pc.a[r], vzp = k < nz - 1 ? zp.a[r] : 2.0 * V - pc.a[r];
      st4<T>(E4 + 4 * (c0 + r), (T)(-(xp - xm) * inv2h), (T)(-(yp.a[r] - ym.a[r]) * inv2h),
             (T)(-(vzp - vzm) * inv2h), (T)0);
    }
  }
}

// One component of the packed field, as double.
template <typename T>
__global__ void k_component(const T* E4, int a, double* out, uint32_t n) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    out[c] = (double)E4[4 * (size_t)c + a];
}

inline int blocks(uint64_t n, int max_blocks = 16384) {
  uint64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > (uint64_t)max_blocks) b = max_blocks;
  return (int)b;
}

}  // namespace

// ---- host side ------------------------------------------------------------------------

struct FieldState {
  int nlev = 0;
  Level lev[kMaxLevels];
  double* phi = nullptr;
  double* b = nullptr;
  void* E[2] = {nullptr, nullptr};  // packed (Ex, Ey, Ez, 0) per cell; E[cur] holds the latest
  int cur = 0;        // E[cur] holds the latest field
  void* sig = nullptr;
  void* ne = nullptr;
  double* norms = nullptr;   // device: ||b||^2, ||r||^2, then per-block partials
  double* host_norms = nullptr;    // mapped pinned host memory: ||b||^2, ||r||^2, sequence
  double* host_norms_dev = nullptr;  // its device address
  unsigned long long seq_expect = 0;  // notifications the host has waited for
  double* phi_prev = nullptr;  // converged potential of the previous step
  bool have_prev = false;
  bool split = false;  // finest level in split red-black order (nx even, more than one level)
  bool seg = false;    // finest-level kernels over 8-cell row segments (nx % 8 == 0, more than one level)
  // per level: split red-black order, and 8-cell row-segment kernels.  The finest level
  // as above; a coarser level (not the coarsest) with nx % 8 == 0 and more than
  // kSmallLevel cells takes both when the finest level is split.
  bool lsplit[kMaxLevels] = {};
  bool lseg[kMaxLevels] = {};
  bool graph_failed = false;
  hipGraphExec_t graph_exec = nullptr;
  // optional timing of the finest-level smoother launches: event pairs recorded around
  // each launch; while timing is on the cycle runs eagerly (not from the graph)
  static constexpr int kMaxTimed = 64;
  hipEvent_t sm_ev[2 * kMaxTimed] = {};
  int sm_n = 0;              // event pairs recorded by the cycle being enqueued
  int sm_pending = 0;        // pairs recorded by the last enqueued cycle, unread
  bool timing = false;
};

static int build_levels(const itokmc_grid_desc* d, int dims[kMaxLevels][3]) {
  int nl = 0;
  int nx = d->nx, ny = d->ny, nz = d->nz;
  for (;;) {
    dims[nl][0] = nx; dims[nl][1] = ny; dims[nl][2] = nz;
    ++nl;
    const int mn = nx < ny ? (nx < nz ? nx : nz) : (ny < nz ? ny : nz);
    if (nl == kMaxLevels || mn < 4 || (nx | ny | nz) & 1) break;
    nx /= 2; ny /= 2; nz /= 2;
  }
  return nl;
}

size_t field_bytes(const itokmc_grid_desc* d) {
  if (d->field_mode != ITOKMC_FIELD_POISSON) return 0;
  const size_t T = d->precision == ITOKMC_FP64 ? 8 : 4;
  const size_t n = (size_t)d->nx * d->ny * d->nz;
  int dims[kMaxLevels][3];
  const int nl = build_levels(d, dims);
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t npart = (size_t)kRedBlocks > (n + 255) / 256 ? (size_t)kRedBlocks : (n + 255) / 256;
  size_t total = al(n * 8) * 3 + al(n * 4 * T) * 2 + al(n * 8) * 2 + al(8 * (8 + npart));
  for (int l = 0; l < nl; ++l) total += 3 * al((size_t)dims[l][0] * dims[l][1] * dims[l][2] * T);
  return total;
}

static FieldState* fs(itokmc_ctx* ctx) { return reinterpret_cast<FieldState*>(ctx->field_state); }

int field_init(itokmc_ctx* ctx, char* base) {
  const itokmc_grid_desc* d = &ctx->d;
  int dims[kMaxLevels][3];
  const int nl = build_levels(d, dims);
  const uint64_t bottom = (uint64_t)dims[nl - 1][0] * dims[nl - 1][1] * dims[nl - 1][2];
  if (bottom > (uint64_t)kBottomMaxCells)
    return set_error(ctx, ITOKMC_EINVAL, "grid cannot be coarsened to <= %d cells (dims must be even)",
                     kBottomMaxCells);
  FieldState* F = new FieldState();
  const size_t T = d->precision == ITOKMC_FP64 ? 8 : 4;
  const size_t n = ctx->ncell;
  auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
  char* p = base;
  F->phi = (double*)p; p += al(n * 8);
  F->b = (double*)p; p += al(n * 8);
  F->phi_prev = (double*)p; p += al(n * 8);
  for (int s = 0; s < 2; ++s)
    { F->E[s] = p; p += al(n * 4 * T); }
  F->sig = p; p += al(n * 8);  // deposit accumulators (8 bytes in either precision)
  F->ne = p; p += al(n * 8);
  const size_t npart = (size_t)kRedBlocks > (n + 255) / 256 ? (size_t)kRedBlocks : (n + 255) / 256;
  F->norms = (double*)p; p += al(8 * (8 + npart));
  F->nlev = nl;
  F->seg = nl > 1 && d->nx % 8 == 0;
  for (int l = 0; l < nl; ++l) {
    Level& L = F->lev[l];
    L.nx = dims[l][0]; L.ny = dims[l][1]; L.nz = dims[l][2];
    L.n = (uint32_t)((size_t)L.nx * L.ny * L.nz);
    L.u = p; p += al(L.n * T);
    L.f = p; p += al(L.n * T);
    L.eps = p; p += al(L.n * T);
  }
  hipError_t e = hipHostMalloc((void**)&F->host_norms, 64, hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) {
    for (int i = 0; i < 8; ++i) F->host_norms[i] = 0.0;
    e = hipHostGetDevicePointer((void**)&F->host_norms_dev, F->host_norms, 0);
  }
  if (e == hipSuccess) e = hipMemsetAsync(F->norms, 0, 8 * sizeof(double), ctx->s);
  if (e == hipSuccess) e = hipMemsetAsync(F->phi, 0, n * 8, ctx->s);
  for (int s = 0; s < 2 && e == hipSuccess; ++s)
    e = hipMemsetAsync(F->E[s], 0, n * 4 * T, ctx->s);
  if (e != hipSuccess) {
    delete F;
    return check_hip(ctx, e, "field init");
  }
  ctx->field_state = F;
  return ITOKMC_OK;
}

// Drop the captured cycle (its launch parameters depend on the tuning).
void field_reset_graph(itokmc_ctx* ctx) {
  FieldState* F = fs(ctx);
  if (!F) return;
  if (F->graph_exec) (void)hipGraphExecDestroy(F->graph_exec);
  F->graph_exec = nullptr;
  F->graph_failed = false;
}

// Turn timing of the finest-level smoother on or off (the cycle graph is rebuilt).
void field_set_timing(itokmc_ctx* ctx, bool on) {
  FieldState* F = fs(ctx);
  if (!F || F->timing == on) return;
  (void)hipStreamSynchronize(ctx->s);
  if (on && !F->sm_ev[0])
    for (int i = 0; i < 2 * FieldState::kMaxTimed; ++i) (void)hipEventCreate(&F->sm_ev[i]);
  F->timing = on;
  F->sm_pending = 0;
}

void field_destroy(itokmc_ctx* ctx) {
  FieldState* F = fs(ctx);
  if (!F) return;
  for (int i = 0; i < 2 * FieldState::kMaxTimed; ++i)
    if (F->sm_ev[i]) (void)hipEventDestroy(F->sm_ev[i]);
  if (F->host_norms) (void)hipHostFree(F->host_norms);
  if (F->graph_exec) (void)hipGraphExecDestroy(F->graph_exec);
  delete F;
  ctx->field_state = nullptr;
}

static Coef coef(const itokmc_ctx* ctx) {
  return Coef{ctx->c.mu_a, ctx->c.mu_E0, ctx->c.mu_b, ctx->c.E_floor, ctx->c.D};
}

// Blocks of 256 threads for one thread per 8-cell row segment of an nx x ny x nz level.
static int seg_blocks(int nx, int ny, int nz) {
  const uint64_t n = (uint64_t)(nx >> 3) * ny * nz;
  return (int)((n + 255) / 256);
}

static dim3 row_grid(int half_nx, int ny, int nz) {
  return dim3((unsigned)((half_nx + 127) / 128), (unsigned)ny, (unsigned)nz);
}

// One colour sweep at level l (the finest level in split order when F->split); the
// finest level's launches are bracketed by event pairs when timing is on.
template <typename T>
static void smooth(FieldState* F, int l, hipStream_t s, int color, bool from_zero = false) {
  Level& L = F->lev[l];
  const dim3 gs = row_grid((L.nx + 1) / 2, L.ny, L.nz);
  T* u = (T*)L.u;
  const T* f = (const T*)L.f;
  const T* ep = (const T*)L.eps;
  if (l > 0) {
    if (F->lsplit[l])
      k_smooth_seg<T, false><<<seg_blocks(L.nx, L.ny, L.nz), 256, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
    else
      k_smooth_rb<T, false><<<gs, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
    return;
  }
  const bool timed = F->timing && F->sm_n < FieldState::kMaxTimed;  // eager cycles only
  if (timed) (void)hipEventRecord(F->sm_ev[2 * F->sm_n], s);
  if (F->split && F->seg && from_zero)
    k_smooth_seg<T, true, true><<<seg_blocks(L.nx, L.ny, L.nz), 256, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
  else if (F->split && F->seg)
    k_smooth_seg<T, true><<<seg_blocks(L.nx, L.ny, L.nz), 256, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
  else if (F->split)
    k_smooth_split<T><<<gs, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
  else
    k_smooth_rb<T, true><<<gs, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
  if (timed) (void)hipEventRecord(F->sm_ev[2 * F->sm_n + 1], s);
  if (timed) ++F->sm_n;
}

// from_zero: the level's correction is zero on entry and not stored (first sweeps of a
// refinement cycle on the finest level with the row-segment smoother).
template <typename T>
static void smooth_sweeps(FieldState* F, int l, hipStream_t s, int count, bool from_zero = false) {
  Level& L = F->lev[l];
  if (l > 0 && L.n <= kSmallLevel) {
    if (count > 0)
      k_sweeps_small<T><<<1, 1024, 0, s>>>((T*)L.u, (const T*)L.f, (const T*)L.eps, L.nx, L.ny, L.nz, count);
    return;
  }
  for (int it = 0; it < count; ++it) {
    smooth<T>(F, l, s, 0, from_zero && it == 0);
    smooth<T>(F, l, s, 1);
  }
}

static bool zero_free_start(const itokmc_ctx* ctx, const FieldState* F) {
  return F->split && F->seg && ctx->tune.mg_pre >= 1;
}

static int bottom_count(const itokmc_ctx* ctx, const Level& L) {
  int mx = L.nx > L.ny ? L.nx : L.ny;
  mx = mx > L.nz ? mx : L.nz;
  return ctx->tune.bottom_sweeps > 0 ? ctx->tune.bottom_sweeps : 4 * mx + 16;
}

// V-cycle from level l.
template <typename T>
static void vcycle(itokmc_ctx* ctx, FieldState* F, int l, hipStream_t s) {
  Level& L = F->lev[l];
  T* u = (T*)L.u;
  const T* f = (const T*)L.f;
  const T* ep = (const T*)L.eps;
  if (l == F->nlev - 1) {
    if (small_fits_lds<T>(L.n))
      launch_small_lds<T>(s, L.n, u, f, ep, L.nx, L.ny, L.nz, bottom_count(ctx, L), true, nullptr, nullptr,
                          nullptr, 0, 0, 0);
    else
      k_bottom<T><<<1, 1024, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, bottom_count(ctx, L));
    return;
  }
  Level& C = F->lev[l + 1];
  if (l > 0 && L.n <= kSmallLevel && small_fits_lds<T>(L.n)) {
    // natural order (small levels are never split): smoothing from the zero
    // correction that every restriction leaves, and restriction; the coarser cycle;
    // prolongation and smoothing
    launch_small_lds<T>(s, L.n, u, f, ep, L.nx, L.ny, L.nz, ctx->tune.mg_pre, true, nullptr, (T*)C.f,
                        (T*)C.u, C.nx, C.ny, C.nz);
    vcycle<T>(ctx, F, l + 1, s);
    launch_small_lds<T>(s, L.n, u, f, ep, L.nx, L.ny, L.nz, ctx->tune.mg_post, false, (const T*)C.u,
                        nullptr, nullptr, C.nx, C.ny, C.nz);
    return;
  }
  smooth_sweeps<T>(F, l, s, ctx->tune.mg_pre, l == 0 && zero_free_start(ctx, F));
  const dim3 gr = row_grid(C.nx, C.ny, C.nz), gp = row_grid(L.nx, L.ny, L.nz);
  const int sb = seg_blocks(L.nx, L.ny, L.nz);
  T* fcp = (T*)C.f;
  T* ucp = (T*)C.u;
  const int rg = seg_blocks(L.nx, C.ny, C.nz);
  const bool fs = F->lsplit[l], csp = F->lsplit[l + 1];
  if (F->lseg[l]) {
    if (fs && csp) k_restrict_seg<T, true, true><<<rg, 256, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, fcp, ucp);
    else if (fs) k_restrict_seg<T, true, false><<<rg, 256, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, fcp, ucp);
    else k_restrict_seg<T, false, false><<<rg, 256, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, fcp, ucp);
  } else if (fs) {
    k_restrict3<T, true><<<gr, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, fcp, ucp, C.nx, C.ny);
  } else {
    k_restrict3<T, false><<<gr, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, fcp, ucp, C.nx, C.ny);
  }
  vcycle<T>(ctx, F, l + 1, s);
  const T* ucc = (const T*)C.u;
  if (F->lseg[l]) {
    if (fs && csp) k_prolong_seg<T, true, true><<<sb, 256, 0, s>>>(u, L.nx, L.ny, L.nz, ucc, C.nx, C.ny, C.nz);
    else if (fs) k_prolong_seg<T, true, false><<<sb, 256, 0, s>>>(u, L.nx, L.ny, L.nz, ucc, C.nx, C.ny, C.nz);
    else k_prolong_seg<T, false, false><<<sb, 256, 0, s>>>(u, L.nx, L.ny, L.nz, ucc, C.nx, C.ny, C.nz);
  } else if (fs) {
    k_prolong3<T, true><<<gp, 128, 0, s>>>(u, L.nx, L.ny, L.nz, ucc, C.nx, C.ny, C.nz);
  } else {
    k_prolong3<T, false><<<gp, 128, 0, s>>>(u, L.nx, L.ny, L.nz, ucc, C.nx, C.ny, C.nz);
  }
  smooth_sweeps<T>(F, l, s, ctx->tune.mg_post);
}

// Wait for the next residual-norm notification (k_sum_notify) by polling the mapped
// host word; after a fraction of a second without it (a failed launch), synchronise the stream,
// which reports the error.  While the smoother is being timed the stream is
// synchronised instead (its events are read right after).
static hipError_t wait_norms(FieldState* F, hipStream_t s) {
  const unsigned long long want = ++F->seq_expect;
  if (F->timing) return hipStreamSynchronize(s);
  volatile unsigned long long* q = reinterpret_cast<volatile unsigned long long*>(F->host_norms) + 2;
  for (long spin = 0; *q < want; ++spin) {
    if (spin > (1L << 26)) {
      const hipError_t e = hipStreamSynchronize(s);
      if (e != hipSuccess) return e;
      if (*q < want) return hipErrorUnknown;
      break;
    }
  }
  return hipSuccess;
}

// Accumulate the timed finest-level smoother launches of the last cycle (the stream
// has been synchronised).
static void collect_smooth(itokmc_ctx* ctx, FieldState* F) {
  for (int i = 0; i < F->sm_pending; ++i) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, F->sm_ev[2 * i], F->sm_ev[2 * i + 1]) == hipSuccess) {
      ctx->phase_ms[PH_SMOOTH_FINE] += ms;
      ctx->phase_calls[PH_SMOOTH_FINE] += 1;
    }
  }
  F->sm_pending = 0;
}

// Double residual of the finest level into f (working precision) and ||r||^2 into
// norms[1].
template <typename T>
static void residual(FieldState* F, hipStream_t s) {
  Level& L0 = F->lev[0];
  if (F->seg) {
    const uint32_t runs = ((L0.n >> 3) + 255) / 256;
    const int rb = runs < (uint32_t)kResBlocks ? (int)runs : kResBlocks;
    if (F->split)
      k_residual_seg<T, true><<<rb, 256, 0, s>>>(F->phi, F->b, (const T*)L0.eps, L0.nx, L0.ny, L0.nz,
                                                 (T*)L0.f, F->norms + 8);
    else
      k_residual_seg<T, false><<<rb, 256, 0, s>>>(F->phi, F->b, (const T*)L0.eps, L0.nx, L0.ny, L0.nz,
                                                  (T*)L0.f, F->norms + 8);
    k_sum_notify<<<1, 1024, 0, s>>>(F->norms + 8, rb, F->norms + 1, F->norms, F->host_norms_dev,
                                    reinterpret_cast<unsigned long long*>(F->norms + 2));
    return;
  }
  const uint32_t runs = (L0.n + 255) / 256;
  const int rb = runs < (uint32_t)kResBlocks ? (int)runs : kResBlocks;
  if (F->split)
    k_residual_rows<T, true><<<rb, 256, 0, s>>>(F->phi, F->b, (const T*)L0.eps, L0.nx, L0.ny, L0.nz,
                                                (T*)L0.f, F->norms + 8);
  else
    k_residual_rows<T, false><<<rb, 256, 0, s>>>(F->phi, F->b, (const T*)L0.eps, L0.nx, L0.ny, L0.nz,
                                                 (T*)L0.f, F->norms + 8);
  k_sum_notify<<<1, 1024, 0, s>>>(F->norms + 8, rb, F->norms + 1, F->norms, F->host_norms_dev,
                                  reinterpret_cast<unsigned long long*>(F->norms + 2));
}

// One refinement cycle: correction V-cycle from zero, potential update, new double
// residual and its norm.
template <typename T>
static void refine_cycle(itokmc_ctx* ctx, FieldState* F, hipStream_t s) {
  Level& L0 = F->lev[0];
  F->sm_n = 0;
  // the correction starts at zero; the first colour-0 sweep can assume it instead (the
  // colour-1 sweep that follows writes the rest of the level before anything reads it)
  if (!zero_free_start(ctx, F)) k_zero<T><<<blocks(L0.n), 256, 0, s>>>((T*)L0.u, L0.n);
  vcycle<T>(ctx, F, 0, s);
  const dim3 gp = row_grid(L0.nx, L0.ny, L0.nz);
  const int sb = seg_blocks(L0.nx, L0.ny, L0.nz);
  if (F->seg && F->split)
    k_phi_update_seg<T, true><<<sb, 256, 0, s>>>(F->phi, (const T*)L0.u, L0.nx, L0.ny, L0.nz);
  else if (F->seg)
    k_phi_update_seg<T, false><<<sb, 256, 0, s>>>(F->phi, (const T*)L0.u, L0.nx, L0.ny, L0.nz);
  else if (F->split) k_phi_update<T, true><<<gp, 128, 0, s>>>(F->phi, (const T*)L0.u, L0.nx, L0.ny);
  else k_phi_update<T, false><<<gp, 128, 0, s>>>(F->phi, (const T*)L0.u, L0.nx, L0.ny);
  residual<T>(F, s);
}

// Capture one refinement cycle into a HIP graph (on a private stream: the caller's
// stream may be the legacy default stream, which cannot be captured).  The graph holds
// kernel nodes only.  Returns false if capture is unavailable; the caller then runs the
// cycle eagerly.
template <typename T>
static bool capture_cycle(itokmc_ctx* ctx, FieldState* F) {
  if (F->graph_exec) return true;
  if (F->graph_failed) return false;
  hipStream_t cs = nullptr;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { F->graph_failed = true; return false; }
  hipGraph_t g = nullptr;
  bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
  if (ok) {
    refine_cycle<T>(ctx, F, cs);
    ok = hipStreamEndCapture(cs, &g) == hipSuccess && g != nullptr;
  }
  hipGraphExec_t ex = nullptr;
  if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cs);
  (void)hipGetLastError();
  if (!ok) { F->graph_failed = true; return false; }
  F->graph_exec = ex;
  return true;
}

// Solve with the current right-hand side b and fine coefficient lev[0].eps.
template <typename T>
static int solve(itokmc_ctx* ctx, FieldState* F) {
  hipStream_t s = ctx->s;
  Level& L0 = F->lev[0];
  for (int l = 1; l < F->nlev; ++l) {
    Level& Fl = F->lev[l - 1];
    Level& Cl = F->lev[l];
    k_eps_restrict<T><<<blocks(Cl.n), 256, 0, s>>>((const T*)Fl.eps, Fl.nx, Fl.ny, F->lsplit[l - 1] ? 1 : 0,
                                                   (T*)Cl.eps, Cl.nx, Cl.ny, Cl.nz, F->lsplit[l] ? 1 : 0);
  }
  const int maxc = ctx->d.gmg_max_cycles > 0 ? ctx->d.gmg_max_cycles : 50;
  ctx->total_solves += 1;
  residual<T>(F, s);
  const bool graph = ctx->tune.use_graph && !F->timing && capture_cycle<T>(ctx, F);
  for (int cyc = 0;; ++cyc) {
    // every residual launch ends with one notification: wait for this one
    hipError_t e = wait_norms(F, s);
    if (e != hipSuccess) return check_hip(ctx, e, "solve residual");
    collect_smooth(ctx, F);
    const double bn2 = F->host_norms[0], rn2 = F->host_norms[1];
    const double bn = bn2 > 0.0 ? sqrt(bn2) : 1.0;
    ctx->last_relres = sqrt(rn2) / bn;
    ctx->last_cycles = cyc;
    if (sqrt(rn2) <= ctx->d.gmg_rtol * bn) break;
    if (cyc >= maxc)
      return set_error(ctx, ITOKMC_ENOCONV, "field solve: relres %.3e after %d cycles", ctx->last_relres, cyc);
    ctx->total_cycles += 1;
    if (graph) {
      e = hipGraphLaunch(F->graph_exec, s);
      if (e != hipSuccess) return check_hip(ctx, e, "solve graph");
      F->sm_pending = 0;
    } else {
      refine_cycle<T>(ctx, F, s);
      F->sm_pending = F->sm_n;
    }
  }
  return check_hip(ctx, hipGetLastError(), "solve");
}

// Deposit (mode 0 initial / 1 semi-implicit), right-hand side, solve, E into E[next].
template <typename T>
static int deposit_and_solve(itokmc_ctx* ctx, FieldState* F, const StepConst& K, int mode) {
  hipStream_t s = ctx->s;
  const uint32_t n = ctx->ncell;
  const bool split = ctx->tune.fine_layout == 0 && F->nlev > 1;
  if (split != F->split) {
    field_reset_graph(ctx);
    F->split = split;
  }
  for (int l = 0; l < F->nlev; ++l) {
    const Level& L = F->lev[l];
    if (l == 0) {
      F->lsplit[0] = F->split;
      F->lseg[0] = F->seg;
    } else {
      F->lseg[l] = F->lsplit[l] = F->split && l < F->nlev - 1 && L.nx % 8 == 0 && L.n > kSmallLevel;
    }
  }
  phase_begin(ctx, PH_FIELD_PREP);
  using S = typename DepAcc<T>::S;
  k_zero<S><<<blocks(n), 256, 0, s>>>((S*)F->sig, n);
  k_zero<S><<<blocks(n), 256, 0, s>>>((S*)F->ne, n);
  phase_end(ctx, PH_FIELD_PREP);
  const void* Eo = F->E[F->cur];
  phase_begin(ctx, PH_DEPOSIT);  // the deposit kernel alone
  {
    constexpr int L2 = DepTbl<T>::log2n;
    const size_t lds = (size_t)(1 << L2) * (4 + 2 * sizeof(S));
    int g = (int)((ctx->cap + kDepChunk - 1) / kDepChunk);
    g = g < 1 ? 1 : (g > 16384 ? 16384 : g);
    if (ctx->d.shape == ITOKMC_SHAPE_TSC)
      k_field_deposit_lds<T, L2, 1><<<g, 256, lds, s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, Eo,
                                                        coef(ctx), mode, (S*)F->sig, (S*)F->ne,
                                                        (uint32_t)kDepChunk, (T*)ctx->mu_p);
    else
      k_field_deposit_lds<T, L2, 0><<<g, 256, lds, s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, Eo,
                                                        coef(ctx), mode, (S*)F->sig, (S*)F->ne,
                                                        (uint32_t)kDepChunk, (T*)ctx->mu_p);
  }
  phase_end(ctx, PH_DEPOSIT);
  phase_begin(ctx, PH_FIELD_PREP);
  const double sig_scale = mode == 1 ? kE * K.dt / (kEps0 * K.dx * K.dx * K.dx) : 0.0;
  if (mode == 1) {
    k_extrapolate<<<blocks(n), 256, 0, s>>>(F->phi, F->phi_prev, n,
                                           (F->have_prev && ctx->tune.extrapolate) ? 1 : 0);
    F->have_prev = true;
  } else {
    F->have_prev = false;
  }
  k_field_prep<T><<<kRedBlocks, 256, 0, s>>>(K, ctx->nplus, ctx->nminus, (const S*)F->ne,
                                             (const S*)F->sig, sig_scale, ctx->d.V_anode,
                                             F->split ? 1 : 0, ctx->d.shape == ITOKMC_SHAPE_TSC ? 1 : 0,
                                             (T*)F->lev[0].eps, F->b, F->norms + 8);
  k_sum_partials<<<1, 1024, 0, s>>>(F->norms + 8, kRedBlocks, F->norms);
  phase_end(ctx, PH_FIELD_PREP);
  phase_begin(ctx, PH_SOLVE);
  const int rc = solve<T>(ctx, F);
  const int nxt = 1 - F->cur;
  if (ctx->d.nx % 4 == 0)
    k_efield_seg<T><<<blocks(n / 4), 256, 0, s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz, ctx->d.V_anode,
                                                  1.0 / (2.0 * ctx->d.dx), (T*)F->E[nxt]);
  else
    k_efield<T><<<blocks(n), 256, 0, s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz, ctx->d.V_anode,
                                          1.0 / (2.0 * ctx->d.dx), (T*)F->E[nxt]);
  phase_end(ctx, PH_SOLVE);
  return rc ? rc : check_hip(ctx, hipGetLastError(), "field");
}

// Initial field: the solution for the present charge with sigma = 0 (the deposit's mode
// 0 uses neither dt nor the diffusion of K).
template <typename T>
static int ensure_field(itokmc_ctx* ctx, FieldState* F, const StepConst& K) {
  if (ctx->field_valid) return 0;
  const int rc = deposit_and_solve<T>(ctx, F, K, 0);
  if (rc) return rc;
  F->cur = 1 - F->cur;
  ctx->field_valid = true;
  return 0;
}

template <typename T>
static int transport_t(itokmc_ctx* ctx, const StepConst& K) {
  FieldState* F = fs(ctx);
  int rc = ensure_field<T>(ctx, F, K);
  if (rc) return rc;
  rc = deposit_and_solve<T>(ctx, F, K, 1);
  if (rc) return rc;
  const int nxt = 1 - F->cur;
  phase_begin(ctx, PH_FIELD_PUSH);
  // at most 1024 workgroups looping over the particles: 0.375 ms per step at 9.5e6
  // particles against 0.405 ms with 4096 and 0.45 ms with 512
  if (ctx->d.shape == ITOKMC_SHAPE_TSC)
    k_push_field<T, 1><<<blocks(ctx->cap, 1024), 256, 0, ctx->s>>>(
        ctx->bank[ctx->cur], ctx->ctr, ctx->cur, ctx->cellacc, ctx->tiles, K, (const T*)ctx->mu_p, F->E[nxt]);
  else
    k_push_field<T, 0><<<blocks(ctx->cap, 1024), 256, 0, ctx->s>>>(
        ctx->bank[ctx->cur], ctx->ctr, ctx->cur, ctx->cellacc, ctx->tiles, K, (const T*)ctx->mu_p, F->E[nxt]);
  phase_end(ctx, PH_FIELD_PUSH);
  F->cur = nxt;  // E^{k+1} becomes the field of the next step
  if (mobile_ions(ctx)) {
    const hipError_t e = launch_ion_move(ctx, K, F->E[nxt]);
    if (e != hipSuccess) return check_hip(ctx, e, "ions");
  }
  return check_hip(ctx, hipGetLastError(), "field push");
}

int field_transport(itokmc_ctx* ctx, const StepConst& K) {
  return ctx->d.precision == ITOKMC_FP64 ? transport_t<double>(ctx, K) : transport_t<float>(ctx, K);
}

// Largest |E|^2 over the cell centres of the packed (Ex, Ey, Ez, 0) field: one partial
// per workgroup, squares summed in double from the stored components (exact for
// single-precision fields), then the largest partial.  Non-negative doubles order as
// their bit patterns, but plain comparisons suffice here: no atomics.
template <typename T>
__global__ void __launch_bounds__(256) k_emax_partial(const T* E4, uint32_t n, double* part) {
  __shared__ double sh[4];
  double m = 0.0;
#pragma unroll 4
  for (uint32_t c = blockIdx.x * 256u + threadIdx.x; c < n; c += gridDim.x * 256u) {
    const V4<T> e = ld4(E4 + 4 * (size_t)c);
    const double x = (double)e.a[0], y = (double)e.a[1], z = (double)e.a[2];
    m = fmax(m, x * x + y * y + z * z);
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
  if (lane_id() == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmax(fmax(sh[0], sh[1]), fmax(sh[2], sh[3]));
}

__global__ void __launch_bounds__(1024) k_max_partials(const double* part, int n, double* out) {
  __shared__ double sh[16];
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += 1024) m = fmax(m, part[i]);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) m = fmax(m, __shfl_xor(m, d, 64));
  if (lane_id() == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < 16; ++i) r = fmax(r, sh[i]);
    *out = r;
  }
}

template <typename T>
static int field_max_t(itokmc_ctx* ctx, double* Emax) {
  FieldState* F = fs(ctx);
  int rc = ensure_field<T>(ctx, F, make_const(ctx, 0.0));
  if (rc) return rc;
  const uint32_t n = ctx->ncell;
  // at most 2048 workgroups (one resident round of 32 waves per CU); the partials
  // buffer holds max(kRedBlocks, blocks(n)) entries
  const int nb = (int)std::min<size_t>(2048, blocks(n));
  hipStream_t s = ctx->s;
  phase_begin(ctx, PH_EMAX);  // the per-cell pass alone
  k_emax_partial<T><<<nb, 256, 0, s>>>((const T*)F->E[F->cur], n, F->norms + 8);
  phase_end(ctx, PH_EMAX);
  k_max_partials<<<1, 1024, 0, s>>>(F->norms + 8, nb, F->norms + 3);
  double m2 = 0.0;
  hipError_t e = hipMemcpyAsync(&m2, F->norms + 3, sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  rc = check_hip(ctx, e, "field max");
  if (rc) return rc;
  *Emax = sqrt(m2);
  return ITOKMC_OK;
}

int field_max(itokmc_ctx* ctx, double* Emax) {
  if (!fs(ctx)) return set_error(ctx, ITOKMC_EINVAL, "no field state");
  return ctx->d.precision == ITOKMC_FP64 ? field_max_t<double>(ctx, Emax) : field_max_t<float>(ctx, Emax);
}

FieldRates field_rates(itokmc_ctx* ctx) {
  FieldState* F = fs(ctx);
  FieldRates r{};
  if (!F) return r;
  r.E4 = F->E[F->cur];
  r.is_double = ctx->d.precision == ITOKMC_FP64 ? 1 : 0;
  r.mu_a = ctx->c.mu_a; r.mu_E0 = ctx->c.mu_E0; r.mu_b = ctx->c.mu_b; r.E_floor = ctx->c.E_floor;
  r.alpha_A = ctx->c.alpha_A; r.alpha_B = ctx->c.alpha_B; r.eta = ctx->c.eta;
  r.kgamma_ratio = ctx->c.kgamma_ratio;
  r.beta_ep = ctx->c.beta_ep; r.beta_ep_b = ctx->c.beta_ep_b; r.Te_a = ctx->c.Te_a;
  r.Te_b = ctx->c.Te_b; r.beta_np = ctx->c.beta_np;
  r.dV = ctx->d.dx * ctx->d.dx * ctx->d.dx;
  return r;
}

int field_get_phi(itokmc_ctx* ctx, double* host) {
  FieldState* F = fs(ctx);
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (e == hipSuccess) e = copy_on(ctx->s, host, F->phi, (size_t)ctx->ncell * 8, hipMemcpyDeviceToHost);
  return check_hip(ctx, e, "get_field");
}

int field_set_phi(itokmc_ctx* ctx, const double* host) {
  FieldState* F = fs(ctx);
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (e == hipSuccess) e = copy_on(ctx->s, F->phi, host, (size_t)ctx->ncell * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return check_hip(ctx, e, "set_field");
  F->have_prev = false;
  const uint32_t n = ctx->ncell;
  if (ctx->d.precision == ITOKMC_FP64)
    k_efield<double><<<blocks(n), 256, 0, ctx->s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz,
                                                    ctx->d.V_anode, 1.0 / (2.0 * ctx->d.dx),
                                                    (double*)F->E[F->cur]);
  else
    k_efield<float><<<blocks(n), 256, 0, ctx->s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz,
                                                   ctx->d.V_anode, 1.0 / (2.0 * ctx->d.dx),
                                                   (float*)F->E[F->cur]);
  ctx->field_valid = true;
  return check_hip(ctx, hipGetLastError(), "set_field");
}

int field_deposit(itokmc_ctx* ctx, int what, void* dev_out) {
  FieldState* F = fs(ctx);
  const uint32_t n = ctx->ncell;
  if (what == ITOKMC_Q_PHI)
    return check_hip(ctx, hipMemcpyAsync(dev_out, F->phi, (size_t)n * 8, hipMemcpyDeviceToDevice, ctx->s),
                     "deposit phi");
  const int a = what - ITOKMC_Q_EX;
  if (ctx->d.precision == ITOKMC_FP64)
    k_component<double><<<blocks(n), 256, 0, ctx->s>>>((const double*)F->E[F->cur], a, (double*)dev_out, n);
  else
    k_component<float><<<blocks(n), 256, 0, ctx->s>>>((const float*)F->E[F->cur], a, (double*)dev_out, n);
  return check_hip(ctx, hipGetLastError(), "deposit E");
}

// CIC electron density of the current particles (diagnostic query), double atomics.
namespace {
template <typename T, int SH>
__global__ void k_cic_density(Bank a, const Counters* ctr, int which, StepConst K, double inv_dV,
                              double* out) {
  const uint32_t n = min(ctr->n[which], K.cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t w = a.w[i];
    if (!w) continue;
    const uint32_t cell = a.cell[i];
    const int ci = (int)(cell % (uint32_t)K.nx), cj = (int)((cell / (uint32_t)K.nx) % (uint32_t)K.ny);
    const int ck = (int)(cell / ((uint32_t)K.nx * (uint32_t)K.ny));
    const double ox = (double)ctp<T>(a.ox)[i], oy = (double)ctp<T>(a.oy)[i], oz = (double)ctp<T>(a.oz)[i];
    const double q = (double)w * inv_dV;
    if constexpr (SH == 0) {
      int i0, j0, k0;
      double fx, fy, fz;
      tent_axis<double>(ci, ox, K.nx, i0, fx);
      tent_axis<double>(cj, oy, K.ny, j0, fy);
      tent_axis<double>(ck, oz, K.nz, k0, fz);
      cic_add<double>(out, K, i0, j0, k0, fx, fy, fz, q);
    } else {
      const Tsc<double> s = tsc_at<double>(K, ci, cj, ck, ox, oy, oz);
      for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
          for (int aa = 0; aa < 3; ++aa) {
            const double wt = (s.wx[aa] * s.wy[b]) * s.wz[c];
            if (wt == 0.0) continue;
            atomicAdd(&out[(size_t)s.ix[aa] + (size_t)K.nx * ((size_t)s.iy[b] + (size_t)K.ny * s.iz[c])], q * wt);
          }
    }
  }
}
}  // namespace

hipError_t launch_cic_density(itokmc_ctx* ctx, double* out) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(double) * ctx->ncell, ctx->s);
  if (e != hipSuccess) return e;
  StepConst K = make_const(ctx, 0.0);
  const double inv_dV = 1.0 / (ctx->d.dx * ctx->d.dx * ctx->d.dx);
  const bool tsc = ctx->d.shape == ITOKMC_SHAPE_TSC;
  Bank b = ctx->bank[ctx->cur];
  if (ctx->d.precision == ITOKMC_FP64) {
    if (tsc) k_cic_density<double, 1><<<2048, 256, 0, ctx->s>>>(b, ctx->ctr, ctx->cur, K, inv_dV, out);
    else k_cic_density<double, 0><<<2048, 256, 0, ctx->s>>>(b, ctx->ctr, ctx->cur, K, inv_dV, out);
  } else {
    if (tsc) k_cic_density<float, 1><<<2048, 256, 0, ctx->s>>>(b, ctx->ctr, ctx->cur, K, inv_dV, out);
    else k_cic_density<float, 0><<<2048, 256, 0, ctx->s>>>(b, ctx->ctr, ctx->cur, K, inv_dV, out);
  }
  return hipGetLastError();
}

// Space charge of the current state (deposit query): e ((n+ - n-) / dV - n_e) with n_e
// the CIC density written into out by launch_cic_density.
namespace {
__global__ void k_rho_from_density(double* out, const uint32_t* np, const uint32_t* nm, StepConst K,
                                   int tsc, double inv_dV) {
  const uint32_t n = K.ncell;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    double ions = (double)np[c] - (double)nm[c];
    if (tsc) {
      const uint32_t row = c / (uint32_t)K.nx, k = row / (uint32_t)K.ny;
      ions = ion_tsc(np, nm, (int)(c - row * (uint32_t)K.nx), (int)(row - k * (uint32_t)K.ny), (int)k, K.nx,
                     K.ny, K.nz);
    }
    out[c] = kE * (ions * inv_dV - out[c]);
  }
}
}  // namespace

hipError_t launch_rho(itokmc_ctx* ctx, double* out) {
  hipError_t e = launch_cic_density(ctx, out);
  if (e != hipSuccess) return e;
  const double inv_dV = 1.0 / (ctx->d.dx * ctx->d.dx * ctx->d.dx);
  const int tsc = ctx->d.shape == ITOKMC_SHAPE_TSC ? 1 : 0;
  k_rho_from_density<<<blocks(ctx->ncell), 256, 0, ctx->s>>>(out, ctx->nplus, ctx->nminus, make_const(ctx, 0.0),
                                                            tsc, inv_dV);
  return hipGetLastError();
}

}  // namespace itk
