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

template <typename T>
__device__ __forceinline__ T cic_get(const T* grid, const StepConst& K, int i0, int j0, int k0, T fx,
                                     T fy, T fz) {
  const int nx = K.nx, ny = K.ny, nz = K.nz;
  T acc = (T)0;
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int di = cc & 1, dj = (cc >> 1) & 1, dk = (cc >> 2) & 1;
    const T wt = (di ? fx : (T)1 - fx) * (dj ? fy : (T)1 - fy) * (dk ? fz : (T)1 - fz);
    const int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
    if (wt == (T)0 || ii >= nx || jj >= ny || kk >= nz) continue;
    acc += grid[(size_t)ii + (size_t)nx * ((size_t)jj + (size_t)ny * kk)] * wt;
  }
  return acc;
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
template <> struct NormalsF<float> {
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

// ---- particle passes --------------------------------------------------------------

// Deposit accumulators.  In single precision the node sums are fixed-point integers
// (conductivity weight mu w in units of 2^-32, electron number in units of 2^-28,
// 64-bit), so a sum does not depend on the order of its atomic additions and the field
// of a realization is bit-reproducible; each single-precision contribution converts
// exactly or to within half a unit.  Ranges: 2^31 and 2^35 per node.  Double precision
// sums doubles.
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
  __device__ static S enc0(float a) { return (S)rintf(a * 0x1p32f); }
  __device__ static S enc1(float a) { return (S)rintf(a * 0x1p28f); }
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
// the step, with the normals of the push).
constexpr int kDepChunk = 2048;
constexpr int kDepProbes = 8;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;
template <typename T> struct DepTbl { static constexpr int log2n = 11; };

template <typename T>
__device__ __forceinline__ void tbl_add(uint32_t* keys, typename DepAcc<T>::S* v0,
                                        typename DepAcc<T>::S* v1, uint32_t node, T a, T b,
                                        typename DepAcc<T>::S* g0, typename DepAcc<T>::S* g1) {
  using A = DepAcc<T>;
  constexpr int L2 = DepTbl<T>::log2n;
  constexpr uint32_t mask = (1u << L2) - 1u;
  uint32_t h = (node * 2654435761u) >> (32 - L2);
  for (int probe = 0; probe < kDepProbes; ++probe) {
    uint32_t k = keys[h];
    if (k == kEmptyKey) {
      const uint32_t prev = atomicCAS(&keys[h], kEmptyKey, node);
      k = prev == kEmptyKey ? node : prev;
    }
    if (k == node) {
      if (a != (T)0) atomicAdd(&v0[h], A::enc0(a));
      if (b != (T)0) atomicAdd(&v1[h], A::enc1(b));
      return;
    }
    h = (h + 1u) & mask;
  }
  if (a != (T)0) atomicAdd(&g0[node], A::enc0(a));
  if (b != (T)0) atomicAdd(&g1[node], A::enc1(b));
}

template <typename T>
__device__ __forceinline__ void tbl_cic(uint32_t* keys, typename DepAcc<T>::S* v0,
                                        typename DepAcc<T>::S* v1, const StepConst& K, int i0,
                                        int j0, int k0, T fx, T fy, T fz, T qa, T qb,
                                        typename DepAcc<T>::S* g0, typename DepAcc<T>::S* g1) {
#pragma unroll
  for (int cc = 0; cc < 8; ++cc) {
    const int di = cc & 1, dj = (cc >> 1) & 1, dk = (cc >> 2) & 1;
    const T wt = (di ? fx : (T)1 - fx) * (dj ? fy : (T)1 - fy) * (dk ? fz : (T)1 - fz);
    const int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
    if (wt == (T)0 || ii >= K.nx || jj >= K.ny || kk >= K.nz) continue;
    const uint32_t node = (uint32_t)ii + (uint32_t)K.nx * ((uint32_t)jj + (uint32_t)K.ny * (uint32_t)kk);
    tbl_add<T>(keys, v0, v1, node, qa * wt, qb * wt, g0, g1);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_field_deposit_lds(Bank a, const Counters* ctr, int which,
                                                          StepConst K, const void* Ex,
                                                          const void* Ey, const void* Ez, Coef co,
                                                          int mode, typename DepAcc<T>::S* sig,
                                                          typename DepAcc<T>::S* ne) {
  using S = typename DepAcc<T>::S;
  constexpr int TBL = 1 << DepTbl<T>::log2n;
  extern __shared__ __align__(16) char smem[];
  S* v0 = reinterpret_cast<S*>(smem);
  S* v1 = v0 + TBL;
  uint32_t* keys = reinterpret_cast<uint32_t*>(v1 + TBL);
  const uint32_t n = min(ctr->n[which], K.cap);
  const T diff = (T)K.diff;
  for (uint32_t c0 = blockIdx.x * (uint32_t)kDepChunk; c0 < n; c0 += gridDim.x * (uint32_t)kDepChunk) {
    for (int t = threadIdx.x; t < TBL; t += blockDim.x) {
      keys[t] = kEmptyKey;
      v0[t] = (S)0;
      v1[t] = (S)0;
    }
    __syncthreads();
    const uint32_t c1 = min(c0 + (uint32_t)kDepChunk, n);
    for (uint32_t i = c0 + threadIdx.x; i < c1; i += blockDim.x) {
      const uint32_t w = a.w[i];
      if (!w) continue;
      const uint32_t cell = a.cell[i];
      const int ci = (int)(cell % (uint32_t)K.nx), cj = (int)((cell / (uint32_t)K.nx) % (uint32_t)K.ny),
                ck = (int)(cell / ((uint32_t)K.nx * (uint32_t)K.ny));
      const T o[3] = {tp<T>(a.ox)[i], tp<T>(a.oy)[i], tp<T>(a.oz)[i]};
      int i0, j0, k0;
      T fx, fy, fz;
      tent_axis<T>(ci, o[0], K.nx, i0, fx);
      tent_axis<T>(cj, o[1], K.ny, j0, fy);
      tent_axis<T>(ck, o[2], K.nz, k0, fz);
      if (mode == 0) {
        tbl_cic<T>(keys, v0, v1, K, i0, j0, k0, fx, fy, fz, (T)0, (T)w, sig, ne);
        continue;
      }
      const T e[3] = {cic_get<T>(ctp<T>(Ex), K, i0, j0, k0, fx, fy, fz),
                      cic_get<T>(ctp<T>(Ey), K, i0, j0, k0, fx, fy, fz),
                      cic_get<T>(ctp<T>(Ez), K, i0, j0, k0, fx, fy, fz)};
      const T Em = sqrt(e[0] * e[0] + e[1] * e[1] + e[2] * e[2]);
      const T mu = Mob<T>::mu(co, Em);
      tbl_cic<T>(keys, v0, v1, K, i0, j0, k0, fx, fy, fz, mu * (T)w, (T)0, sig, ne);
      const uint64_t id = a.id[i];
      const uint4 r = philox_block((uint32_t)id, (uint32_t)(id >> 32), K.step, TAG_PUSH, 0, K.key);
      T nr[3];
      NormalsF<T>::get(r, nr);
      tent_axis<T>(ci, o[0] + diff * nr[0], K.nx, i0, fx);
      tent_axis<T>(cj, o[1] + diff * nr[1], K.ny, j0, fy);
      tent_axis<T>(ck, o[2] + diff * nr[2], K.nz, k0, fz);
      tbl_cic<T>(keys, v0, v1, K, i0, j0, k0, fx, fy, fz, (T)0, (T)w, sig, ne);
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
template <typename T>
__global__ void __launch_bounds__(256) k_push_field(Bank a, Counters* ctr, int which,
                                                   unsigned long long* cellacc, uint32_t* tiles,
                                                   StepConst K,
                                                   const void* Eox, const void* Eoy, const void* Eoz,
                                                   const void* Enx, const void* Eny, const void* Enz,
                                                   Coef co) {
  const uint32_t n = min(ctr->n[which], K.cap);
  const T diff = (T)K.diff;
  const T dtdx = (T)(K.dt / K.dx);
  uint64_t out_w = 0, pushed = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t key = kInvalidCell, w = 0;
    if (i < n) w = a.w[i];
    if (w > 0) {
      ++pushed;
      const uint32_t cell = a.cell[i];
      int ci[3] = {(int)(cell % (uint32_t)K.nx), (int)((cell / (uint32_t)K.nx) % (uint32_t)K.ny),
                   (int)(cell / ((uint32_t)K.nx * (uint32_t)K.ny))};
      T o[3] = {tp<T>(a.ox)[i], tp<T>(a.oy)[i], tp<T>(a.oz)[i]};
      int i0, j0, k0;
      T fx, fy, fz;
      tent_axis<T>(ci[0], o[0], K.nx, i0, fx);
      tent_axis<T>(ci[1], o[1], K.ny, j0, fy);
      tent_axis<T>(ci[2], o[2], K.nz, k0, fz);
      const T eo[3] = {cic_get<T>(ctp<T>(Eox), K, i0, j0, k0, fx, fy, fz),
                       cic_get<T>(ctp<T>(Eoy), K, i0, j0, k0, fx, fy, fz),
                       cic_get<T>(ctp<T>(Eoz), K, i0, j0, k0, fx, fy, fz)};
      const T en[3] = {cic_get<T>(ctp<T>(Enx), K, i0, j0, k0, fx, fy, fz),
                       cic_get<T>(ctp<T>(Eny), K, i0, j0, k0, fx, fy, fz),
                       cic_get<T>(ctp<T>(Enz), K, i0, j0, k0, fx, fy, fz)};
      const T mu = Mob<T>::mu(co, sqrt(eo[0] * eo[0] + eo[1] * eo[1] + eo[2] * eo[2]));
      const uint64_t id = a.id[i];
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
    const uint64_t old = run_add(cellacc, key, key != kInvalidCell ? ((1ull << 32) | w) : 0ull);
    mark_tile(tiles, key, old);
    if (key != kInvalidCell) a.rank[i] = (uint32_t)(old >> 32);
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
                                                   double sig_scale, double V, int split, T* eps,
                                                   double* b, double* partial) {
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
      const double rho_units = (double)nplus[c] - (double)nminus[c] - DepAcc<T>::dec1(ne[c]);
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
__global__ void k_eps_restrict(const T* ef, int fnx, int fny, int fsplit, T* ec, int cnx, int cny, int cnz) {
  const uint32_t n = (uint32_t)cnx * cny * cnz;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int i = c % cnx, j = (c / cnx) % cny, k = c / (cnx * cny);
    double s = 0.0;
    for (int d = 0; d < 8; ++d) {
      const int fi = 2 * i + (d & 1), fj = 2 * j + ((d >> 1) & 1), fk = 2 * k + (d >> 2);
      s += (double)ef[fsplit ? pos_of<true>(fi, fj, fk, fnx, fny) : pos_of<false>(fi, fj, fk, fnx, fny)];
    }
    ec[c] = (T)(s * 0.125);
  }
}

// Harmonic mean for the smoother: exact in double; fast reciprocal in single precision
// (the smoother only has to reduce the error; the double residual of the refinement
// loop defines the solution).
__device__ __forceinline__ double hmean_s(double a, double b) { return 2.0 * a * b / (a + b); }
__device__ __forceinline__ float hmean_s(float a, float b) { return __fdividef(2.0f * a * b, a + b); }

// Operator of the scaled system at one cell (homogeneous boundary values): sum over
// faces of beta (u_c - u_nb), beta the harmonic mean of the two cells' coefficients,
// plus 2 eps_c u_c on the Dirichlet z faces; x and y faces are Neumann.  Returned as
// the diagonal and the neighbour sum.  Working-precision row through value accessors
// a(dx, dy, dz) of the correction and of the coefficient at the neighbour (dx, dy, dz)
// of cell (i, j, k), so the smoothers reading HBM and reading LDS share one arithmetic
// order.  All thirteen values are read before any arithmetic (offsets clamped to the
// cell itself on the domain faces), so their loads are in flight together; a face
// outside the domain then contributes nothing, or the Dirichlet term, in the same
// order as the faces are listed.
template <typename T, typename UA, typename EA>
__device__ __forceinline__ void stencil_acc(UA ua, EA ea, int nx, int ny, int nz, int i, int j, int k,
                                            T& diag, T& offsum) {
  const bool in[6] = {i > 0, i < nx - 1, j > 0, j < ny - 1, k > 0, k < nz - 1};
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

// Operator row for the double residual with the face coefficients computed exactly as
// the smoother computes them (single-precision harmonic means in FP32 mode, exact double
// in FP64 mode), accumulated in double; the potential in natural order, the
// coefficient through its level's positions `at`.
template <typename T, typename AT>
__device__ __forceinline__ void stencil_r(const double* u, const T* eps, AT at, int nx, int ny, int nz,
                                          int i, int j, int k, size_t c, double& diag, double& offsum) {
  const ptrdiff_t sy = (ptrdiff_t)nx, sz = (ptrdiff_t)nx * ny;
  const bool in[6] = {i > 0, i < nx - 1, j > 0, j < ny - 1, k > 0, k < nz - 1};
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

// Logical (x, y, z) block of a 3-D grid after the XCD remap.
__device__ __forceinline__ void xcd_block3(int& bx, int& by, int& bz) {
  const uint32_t nb = gridDim.x * gridDim.y * gridDim.z;
  const uint32_t lin = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const uint32_t l = xcd_block(lin, nb);
  bx = (int)(l % gridDim.x);
  by = (int)((l / gridDim.x) % gridDim.y);
  bz = (int)(l / (gridDim.x * gridDim.y));
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
  const size_t c = (size_t)i + (size_t)nx * ((size_t)j + (size_t)ny * k);
  T d, s;
  stencil_s<T>(u, eps, nx, ny, nz, i, j, k, c, d, s);
  u[c] = (f[c] + s) / d;
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
  u[at.own] = (f[at.own] + s) / d;
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

// Coarse right-hand side (sum of the 8 child residuals / 2) and zero coarse correction;
// grid (x: coarse row, y: cj, z: ck); the fine level in split order if kSplit.
template <typename T, bool kSplit>
__global__ void __launch_bounds__(128) k_restrict3(const T* u, const T* f, const T* eps, int nx, int ny,
                                                  int nz, T* fc, T* uc, int cnx, int cny) {
  int bx, cj, ck;
  xcd_block3(bx, cj, ck);
  const int ci = bx * blockDim.x + threadIdx.x;
  if (ci >= cnx) return;
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

// Trilinear prolongation of the coarse correction onto cell centres: along each axis
// the nearer coarse centre weighs 3/4 and the farther 1/4; coarse ghost values mirror
// the cell on the Neumann x and y faces and negate it on the homogeneous Dirichlet z
// faces.  (Second-order transfer: with cell-averaged restriction the transfer orders
// then exceed the order of the operator.)
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
  u[(size_t)p + (size_t)nx * ((size_t)j + (size_t)ny * k)] += acc;
}

// Coarsest level: red-black sweeps from zero inside one workgroup.
template <typename T>
__global__ void __launch_bounds__(1024) k_bottom(T* u, const T* f, const T* eps, int nx, int ny, int nz,
                                                int sweeps) {
  const int n = nx * ny * nz;
  for (int c = threadIdx.x; c < n; c += blockDim.x) u[c] = (T)0;
  __syncthreads();
  for (int s = 0; s < sweeps; ++s)
    for (int color = 0; color < 2; ++color) {
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
        if (((i + j + k) & 1) != color) continue;
        T d, sm;
        stencil_s<T>(u, eps, nx, ny, nz, i, j, k, (size_t)c, d, sm);
        u[c] = (f[c] + sm) / d;
      }
      __syncthreads();
    }
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

template <typename T>
__global__ void k_efield(const double* phi, int nx, int ny, int nz, double V, double inv2h, T* Ex, T* Ey,
                         T* Ez) {
  const uint32_t n = (uint32_t)nx * ny * nz;
  const size_t sy = (size_t)nx, sz = (size_t)nx * ny;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    const double pc = phi[c];
    const double xm = i > 0 ? phi[c - 1] : pc, xp = i < nx - 1 ? phi[c + 1] : pc;
    const double ym = j > 0 ? phi[c - sy] : pc, yp = j < ny - 1 ? phi[c + sy] : pc;
    const double zm = k > 0 ? phi[c - sz] : -pc, zp = k < nz - 1 ? phi[c + sz] : 2.0 * V - pc;
    Ex[c] = (T)(-(xp - xm) * inv2h);
    Ey[c] = (T)(-(yp - ym) * inv2h);
    Ez[c] = (T)(-(zp - zm) * inv2h);
  }
}

template <typename T>
__global__ void k_to_double(const T* a, double* out, uint32_t n) {
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x)
    out[c] = (double)a[c];
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
  void* E[2][3] = {{nullptr, nullptr, nullptr}, {nullptr, nullptr, nullptr}};
  int cur = 0;        // E[cur] holds the latest field
  void* sig = nullptr;
  void* ne = nullptr;
  double* norms = nullptr;   // device: ||b||^2, ||r||^2, then per-block partials
  double* host_norms = nullptr;
  double* phi_prev = nullptr;  // converged potential of the previous step
  bool have_prev = false;
  bool split = false;  // finest level in split red-black order (nx even, more than one level)
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
  size_t total = al(n * 8) * 3 + al(n * T) * 6 + al(n * 8) * 2 + al(8 * (8 + npart));
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
    for (int a = 0; a < 3; ++a) { F->E[s][a] = p; p += al(n * T); }
  F->sig = p; p += al(n * 8);  // deposit accumulators (8 bytes in either precision)
  F->ne = p; p += al(n * 8);
  const size_t npart = (size_t)kRedBlocks > (n + 255) / 256 ? (size_t)kRedBlocks : (n + 255) / 256;
  F->norms = (double*)p; p += al(8 * (8 + npart));
  F->nlev = nl;
  for (int l = 0; l < nl; ++l) {
    Level& L = F->lev[l];
    L.nx = dims[l][0]; L.ny = dims[l][1]; L.nz = dims[l][2];
    L.n = (uint32_t)((size_t)L.nx * L.ny * L.nz);
    L.u = p; p += al(L.n * T);
    L.f = p; p += al(L.n * T);
    L.eps = p; p += al(L.n * T);
  }
  hipError_t e = hipHostMalloc((void**)&F->host_norms, 64, hipHostMallocDefault);
  if (e == hipSuccess) e = hipMemsetAsync(F->phi, 0, n * 8, ctx->s);
  for (int s = 0; s < 2 && e == hipSuccess; ++s)
    for (int a = 0; a < 3 && e == hipSuccess; ++a) e = hipMemsetAsync(F->E[s][a], 0, n * T, ctx->s);
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

static dim3 row_grid(int half_nx, int ny, int nz) {
  return dim3((unsigned)((half_nx + 127) / 128), (unsigned)ny, (unsigned)nz);
}

// One colour sweep at level l (the finest level in split order when F->split); the
// finest level's launches are bracketed by event pairs when timing is on.
template <typename T>
static void smooth(FieldState* F, int l, hipStream_t s, int color) {
  Level& L = F->lev[l];
  const dim3 gs = row_grid((L.nx + 1) / 2, L.ny, L.nz);
  T* u = (T*)L.u;
  const T* f = (const T*)L.f;
  const T* ep = (const T*)L.eps;
  if (l > 0) {
    k_smooth_rb<T, false><<<gs, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
    return;
  }
  const bool timed = F->timing && F->sm_n < FieldState::kMaxTimed;  // eager cycles only
  if (timed) (void)hipEventRecord(F->sm_ev[2 * F->sm_n], s);
  if (F->split) k_smooth_split<T><<<gs, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
  else k_smooth_rb<T, true><<<gs, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, color);
  if (timed) (void)hipEventRecord(F->sm_ev[2 * F->sm_n + 1], s);
  if (timed) ++F->sm_n;
}

template <typename T>
static void smooth_sweeps(FieldState* F, int l, hipStream_t s, int count) {
  for (int it = 0; it < count; ++it) {
    smooth<T>(F, l, s, 0);
    smooth<T>(F, l, s, 1);
  }
}

template <typename T>
static void vcycle(itokmc_ctx* ctx, FieldState* F, int l, hipStream_t s) {
  Level& L = F->lev[l];
  T* u = (T*)L.u;
  const T* f = (const T*)L.f;
  const T* ep = (const T*)L.eps;
  if (l == F->nlev - 1) {
    int mx = L.nx > L.ny ? L.nx : L.ny;
    mx = mx > L.nz ? mx : L.nz;
    const int bs = ctx->tune.bottom_sweeps > 0 ? ctx->tune.bottom_sweeps : 4 * mx + 16;
    k_bottom<T><<<1, 1024, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, bs);
    return;
  }
  Level& C = F->lev[l + 1];
  smooth_sweeps<T>(F, l, s, ctx->tune.mg_pre);
  const dim3 gr = row_grid(C.nx, C.ny, C.nz), gp = row_grid(L.nx, L.ny, L.nz);
  if (l == 0 && F->split)
    k_restrict3<T, true><<<gr, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, (T*)C.f, (T*)C.u, C.nx, C.ny);
  else
    k_restrict3<T, false><<<gr, 128, 0, s>>>(u, f, ep, L.nx, L.ny, L.nz, (T*)C.f, (T*)C.u, C.nx, C.ny);
  vcycle<T>(ctx, F, l + 1, s);
  if (l == 0 && F->split)
    k_prolong3<T, true><<<gp, 128, 0, s>>>(u, L.nx, L.ny, L.nz, (const T*)C.u, C.nx, C.ny, C.nz);
  else
    k_prolong3<T, false><<<gp, 128, 0, s>>>(u, L.nx, L.ny, L.nz, (const T*)C.u, C.nx, C.ny, C.nz);
  smooth_sweeps<T>(F, l, s, ctx->tune.mg_post);
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
  const uint32_t runs = (L0.n + 255) / 256;
  const int rb = runs < (uint32_t)kResBlocks ? (int)runs : kResBlocks;
  if (F->split)
    k_residual_rows<T, true><<<rb, 256, 0, s>>>(F->phi, F->b, (const T*)L0.eps, L0.nx, L0.ny, L0.nz,
                                                (T*)L0.f, F->norms + 8);
  else
    k_residual_rows<T, false><<<rb, 256, 0, s>>>(F->phi, F->b, (const T*)L0.eps, L0.nx, L0.ny, L0.nz,
                                                 (T*)L0.f, F->norms + 8);
  k_sum_partials<<<1, 1024, 0, s>>>(F->norms + 8, rb, F->norms + 1);
}

// One refinement cycle: correction V-cycle from zero, potential update, new double
// residual and its norm.
template <typename T>
static void refine_cycle(itokmc_ctx* ctx, FieldState* F, hipStream_t s) {
  Level& L0 = F->lev[0];
  F->sm_n = 0;
  k_zero<T><<<blocks(L0.n), 256, 0, s>>>((T*)L0.u, L0.n);
  vcycle<T>(ctx, F, 0, s);
  const dim3 gp = row_grid(L0.nx, L0.ny, L0.nz);
  if (F->split) k_phi_update<T, true><<<gp, 128, 0, s>>>(F->phi, (const T*)L0.u, L0.nx, L0.ny);
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
    k_eps_restrict<T><<<blocks(Cl.n), 256, 0, s>>>((const T*)Fl.eps, Fl.nx, Fl.ny,
                                                   (l == 1 && F->split) ? 1 : 0, (T*)Cl.eps, Cl.nx,
                                                   Cl.ny, Cl.nz);
  }
  const int maxc = ctx->d.gmg_max_cycles > 0 ? ctx->d.gmg_max_cycles : 50;
  ctx->total_solves += 1;
  residual<T>(F, s);
  const bool graph = ctx->tune.use_graph && !F->timing && capture_cycle<T>(ctx, F);
  for (int cyc = 0;; ++cyc) {
    hipError_t e = hipMemcpyAsync(F->host_norms, F->norms, 16, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
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
  phase_begin(ctx, PH_FIELD_PREP);
  using S = typename DepAcc<T>::S;
  k_zero<S><<<blocks(n), 256, 0, s>>>((S*)F->sig, n);
  k_zero<S><<<blocks(n), 256, 0, s>>>((S*)F->ne, n);
  phase_end(ctx, PH_FIELD_PREP);
  void* const* Eo = F->E[F->cur];
  phase_begin(ctx, PH_DEPOSIT);  // the deposit kernel alone
  {
    constexpr int TBL = 1 << DepTbl<T>::log2n;
    const size_t lds = (size_t)TBL * (4 + 2 * sizeof(S));
    int g = (int)((ctx->cap + kDepChunk - 1) / kDepChunk);
    g = g < 1 ? 1 : (g > 4096 ? 4096 : g);
    k_field_deposit_lds<T><<<g, 256, lds, s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, Eo[0], Eo[1],
                                               Eo[2], coef(ctx), mode, (S*)F->sig, (S*)F->ne);
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
                                             F->split ? 1 : 0, (T*)F->lev[0].eps, F->b, F->norms + 8);
  k_sum_partials<<<1, 1024, 0, s>>>(F->norms + 8, kRedBlocks, F->norms);
  phase_end(ctx, PH_FIELD_PREP);
  phase_begin(ctx, PH_SOLVE);
  const int rc = solve<T>(ctx, F);
  const int nxt = 1 - F->cur;
  k_efield<T><<<blocks(n), 256, 0, s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz, ctx->d.V_anode,
                                        1.0 / (2.0 * ctx->d.dx), (T*)F->E[nxt][0], (T*)F->E[nxt][1],
                                        (T*)F->E[nxt][2]);
  phase_end(ctx, PH_SOLVE);
  return rc ? rc : check_hip(ctx, hipGetLastError(), "field");
}

template <typename T>
static int transport_t(itokmc_ctx* ctx, const StepConst& K) {
  FieldState* F = fs(ctx);
  if (!ctx->field_valid) {
    // initial field: the solution for the present charge with sigma = 0
    const int rc = deposit_and_solve<T>(ctx, F, K, 0);
    if (rc) return rc;
    F->cur = 1 - F->cur;
    ctx->field_valid = true;
  }
  const int rc = deposit_and_solve<T>(ctx, F, K, 1);
  if (rc) return rc;
  const int nxt = 1 - F->cur;
  phase_begin(ctx, PH_FIELD_PUSH);
  k_push_field<T><<<blocks(ctx->cap, 4096), 256, 0, ctx->s>>>(
      ctx->bank[ctx->cur], ctx->ctr, ctx->cur, ctx->cellacc, ctx->tiles, K, F->E[F->cur][0], F->E[F->cur][1],
      F->E[F->cur][2], F->E[nxt][0], F->E[nxt][1], F->E[nxt][2], coef(ctx));
  phase_end(ctx, PH_FIELD_PUSH);
  F->cur = nxt;  // E^{k+1} becomes the field of the next step
  return check_hip(ctx, hipGetLastError(), "field push");
}

int field_transport(itokmc_ctx* ctx, const StepConst& K) {
  return ctx->d.precision == ITOKMC_FP64 ? transport_t<double>(ctx, K) : transport_t<float>(ctx, K);
}

FieldRates field_rates(itokmc_ctx* ctx) {
  FieldState* F = fs(ctx);
  FieldRates r{};
  if (!F) return r;
  for (int a = 0; a < 3; ++a) r.E[a] = F->E[F->cur][a];
  r.is_double = ctx->d.precision == ITOKMC_FP64 ? 1 : 0;
  r.mu_a = ctx->c.mu_a; r.mu_E0 = ctx->c.mu_E0; r.mu_b = ctx->c.mu_b; r.E_floor = ctx->c.E_floor;
  r.alpha_A = ctx->c.alpha_A; r.alpha_B = ctx->c.alpha_B; r.eta = ctx->c.eta;
  r.kgamma_ratio = ctx->c.kgamma_ratio;
  return r;
}

int field_get_phi(itokmc_ctx* ctx, double* host) {
  FieldState* F = fs(ctx);
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (e == hipSuccess) e = hipMemcpy(host, F->phi, (size_t)ctx->ncell * 8, hipMemcpyDeviceToHost);
  return check_hip(ctx, e, "get_field");
}

int field_set_phi(itokmc_ctx* ctx, const double* host) {
  FieldState* F = fs(ctx);
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (e == hipSuccess) e = hipMemcpy(F->phi, host, (size_t)ctx->ncell * 8, hipMemcpyHostToDevice);
  if (e != hipSuccess) return check_hip(ctx, e, "set_field");
  F->have_prev = false;
  const uint32_t n = ctx->ncell;
  if (ctx->d.precision == ITOKMC_FP64)
    k_efield<double><<<blocks(n), 256, 0, ctx->s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz,
                                                    ctx->d.V_anode, 1.0 / (2.0 * ctx->d.dx),
                                                    (double*)F->E[F->cur][0], (double*)F->E[F->cur][1],
                                                    (double*)F->E[F->cur][2]);
  else
    k_efield<float><<<blocks(n), 256, 0, ctx->s>>>(F->phi, ctx->d.nx, ctx->d.ny, ctx->d.nz,
                                                   ctx->d.V_anode, 1.0 / (2.0 * ctx->d.dx),
                                                   (float*)F->E[F->cur][0], (float*)F->E[F->cur][1],
                                                   (float*)F->E[F->cur][2]);
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
    k_to_double<double><<<blocks(n), 256, 0, ctx->s>>>((const double*)F->E[F->cur][a], (double*)dev_out, n);
  else
    k_to_double<float><<<blocks(n), 256, 0, ctx->s>>>((const float*)F->E[F->cur][a], (double*)dev_out, n);
  return check_hip(ctx, hipGetLastError(), "deposit E");
}

// CIC electron density of the current particles (diagnostic query), double atomics.
namespace {
template <typename T>
__global__ void k_cic_density(Bank a, const Counters* ctr, int which, StepConst K, double inv_dV,
                              double* out) {
  const uint32_t n = min(ctr->n[which], K.cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t w = a.w[i];
    if (!w) continue;
    const uint32_t cell = a.cell[i];
    int i0, j0, k0;
    double fx, fy, fz;
    tent_axis<double>((int)(cell % (uint32_t)K.nx), (double)ctp<T>(a.ox)[i], K.nx, i0, fx);
    tent_axis<double>((int)((cell / (uint32_t)K.nx) % (uint32_t)K.ny), (double)ctp<T>(a.oy)[i], K.ny, j0, fy);
    tent_axis<double>((int)(cell / ((uint32_t)K.nx * (uint32_t)K.ny)), (double)ctp<T>(a.oz)[i], K.nz, k0, fz);
    cic_add<double>(out, K, i0, j0, k0, fx, fy, fz, (double)w * inv_dV);
  }
}
}  // namespace

hipError_t launch_cic_density(itokmc_ctx* ctx, double* out) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(double) * ctx->ncell, ctx->s);
  if (e != hipSuccess) return e;
  StepConst K = make_const(ctx, 0.0);
  const double inv_dV = 1.0 / (ctx->d.dx * ctx->d.dx * ctx->d.dx);
  if (ctx->d.precision == ITOKMC_FP64)
    k_cic_density<double><<<2048, 256, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, inv_dV, out);
  else
    k_cic_density<float><<<2048, 256, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, inv_dV, out);
  return hipGetLastError();
}

}  // namespace itk
