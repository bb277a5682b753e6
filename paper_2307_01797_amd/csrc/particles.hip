// Particle kernels: seeding, the explicit Ito push with fused NGP binning, photon
// transport, the counting sort by cell (scan + scatter) and reductions.
#include <math.h>

#include <algorithm>

#include "device.hpp"
#include "itk.hpp"
#include "poisson.hpp"
#include "push_device.hpp"

namespace itk {

namespace {

constexpr int kBlock = 256;

inline int grid_for(uint64_t n, int per_block = kBlock, int max_blocks = 8192) {
  uint64_t b = (n + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > (uint64_t)max_blocks) b = max_blocks;
  return (int)b;
}

template <typename T>
__device__ __forceinline__ T* as(void* p) { return reinterpret_cast<T*>(p); }

// Store one particle into a bank slot.
template <typename T>
__device__ __forceinline__ void put(const Bank& b, uint32_t q, uint32_t cell, T ox, T oy, T oz,
                                    uint32_t w, uint64_t id) {
  b.cell[q] = cell;
  as<T>(b.ox)[q] = ox;
  as<T>(b.oy)[q] = oy;
  as<T>(b.oz)[q] = oz;
  b.w[q] = w;
  b.id[q] = id;
}

// ---- seeding ---------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) k_seed_gaussian(Bank b, Counters* ctr, int which,
                                                         StepConst k, uint64_t n0, double cx,
                                                         double cy, double cz, double sigma) {
  const int lim[3] = {k.nx, k.ny, k.nz};
  const double c[3] = {cx, cy, cz};
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n0;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = base + threadIdx.x;
    bool keep = false;
    double xi[3];
    if (i < n0) keep = gaussian_seed_point(i, k.key, k.dx, lim, c, sigma, xi);
    const uint32_t q = wave_append(&ctr->n[which], keep ? 1u : 0u);
    if (keep) {
      if (q >= k.cap) {
        atomicOr(&ctr->overflow, 1u);
      } else {
        const double f[3] = {floor(xi[0]), floor(xi[1]), floor(xi[2])};
        const uint32_t cell =
            (uint32_t)f[0] + (uint32_t)k.nx * ((uint32_t)f[1] + (uint32_t)k.ny * (uint32_t)f[2]);
        put<T>(b, q, cell, to_off<T>(xi[0] - f[0]), to_off<T>(xi[1] - f[1]),
               to_off<T>(xi[2] - f[2]), 1u, (1ull << 61) | i);
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_seed_neutral(Bank b, Counters* ctr, int which,
                                                        StepConst k, uint32_t* nplus,
                                                        int n_new, double n_peak, double cx,
                                                        double cy, double cz, double sigma) {
  const double dV = k.dx * k.dx * k.dx;
  for (uint32_t base = blockIdx.x * blockDim.x; base < k.ncell; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    int64_t N = 0;
    if (c < k.ncell) {
      const uint32_t i = c % (uint32_t)k.nx, j = (c / (uint32_t)k.nx) % (uint32_t)k.ny,
                     kk = c / ((uint32_t)k.nx * (uint32_t)k.ny);
      const double x = (i + 0.5) * k.dx - cx, y = (j + 0.5) * k.dx - cy, z = (kk + 0.5) * k.dx - cz;
      const double lam = n_peak * exp(-(x * x + y * y + z * z) / (2.0 * sigma * sigma)) * dV;
      CellStream st;
      st.init(c, 0, TAG_SEED, 1, k.key);
      N = poisson_draw(lam, st);
    }
    const uint32_t M = N > 0 ? (uint32_t)(N < n_new ? N : n_new) : 0u;
    const uint32_t q0 = wave_append(&ctr->n[which], M);
    if (M > 0) {
      const uint32_t i = c % (uint32_t)k.nx, j = (c / (uint32_t)k.nx) % (uint32_t)k.ny,
                     kk = c / ((uint32_t)k.nx * (uint32_t)k.ny);
      (void)i; (void)j; (void)kk;
      const uint32_t wb = (uint32_t)(N / M), wr = (uint32_t)(N % M);
      for (uint32_t s = 0; s < M; ++s) {
        const uint32_t q = q0 + s;
        if (q >= k.cap) { atomicOr(&ctr->overflow, 1u); break; }
        const uint4 r = philox_block(c, s, 0, TAG_SEED, 2, k.key);
        put<T>(b, q, c, (T)u24(r.x), (T)u24(r.y), (T)u24(r.z), wb + (s == 0 ? wr : 0u),
               ((uint64_t)c << 16) | s);
      }
      nplus[c] += (uint32_t)N;
    }
  }
}

// ---- push (uniform prescribed field) with fused NGP binning -------------------------

template <typename T>
__global__ void __launch_bounds__(kBlock) k_push_uniform(Bank a, Counters* ctr, int which,
                                                        unsigned long long* cellacc,
                                                        uint32_t* tiles, StepConst k) {
  if (ctr->halt) return;
  const uint32_t n = min(ctr->n[which], k.cap);
  const T drift[3] = {(T)k.drift[0], (T)k.drift[1], (T)k.drift[2]};
  const T diff = (T)k.diff;
  uint64_t out_w = 0, pushed = 0;
  const int lim[3] = {k.nx, k.ny, k.nz};
  // two particles per thread (a workgroup-sized stride apart, so that loads stay
  // coalesced): both particles' words are requested before either is pushed
  for (uint32_t base = blockIdx.x * blockDim.x * 2u; base < n; base += gridDim.x * blockDim.x * 2u) {
    uint32_t ii[2] = {base + threadIdx.x, base + blockDim.x + threadIdx.x};
    uint32_t w[2] = {0, 0}, cell[2] = {0, 0};
    uint64_t id[2] = {0, 0};
    T o[2][3] = {{(T)0, (T)0, (T)0}, {(T)0, (T)0, (T)0}};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (ii[q] < n) {
        w[q] = a.w[ii[q]];
        cell[q] = a.cell[ii[q]];
        id[q] = a.id[ii[q]];
        o[q][0] = as<T>(a.ox)[ii[q]];
        o[q][1] = as<T>(a.oy)[ii[q]];
        o[q][2] = as<T>(a.oz)[ii[q]];
      }
    }
    uint32_t key[2] = {kInvalidCell, kInvalidCell};
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (w[q] > 0) {
        ++pushed;
        int ci[3];
        cell_ijk(cell[q], k, ci[0], ci[1], ci[2]);
        const bool inside = push_uniform<T>(id[q], k.step, k.key, drift, diff, lim, ci, o[q]);
        if (inside) {
          key[q] = (uint32_t)ci[0] + (uint32_t)k.nx * ((uint32_t)ci[1] + (uint32_t)k.ny * (uint32_t)ci[2]);
          a.cell[ii[q]] = key[q];
          as<T>(a.ox)[ii[q]] = o[q][0];
          as<T>(a.oy)[ii[q]] = o[q][1];
          as<T>(a.oz)[ii[q]] = o[q][2];
        } else {
          out_w += w[q];
          a.w[ii[q]] = 0;
        }
      }
    }
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const uint32_t rank = bin_add(cellacc, key[q], w[q]);
      mark_tile(tiles, key[q], (uint64_t)rank << 32);
      if (key[q] != kInvalidCell) a.rank[ii[q]] = rank;
    }
  }
  out_w = wave_sum64(out_w);
  pushed = wave_sum64(pushed);
  if (lane_id() == 0) {
    if (out_w) atomicAdd(&ctr->outflow, (unsigned long long)out_w);
    if (pushed) atomicAdd(&ctr->pushed, (unsigned long long)pushed);
  }
}

// Bin the current particles without moving them (after seeding or set_state).
__global__ void __launch_bounds__(kBlock) k_count(Bank a, Counters* ctr, int which,
                                                 unsigned long long* cellacc, uint32_t* tiles,
                                                 uint32_t cap) {
  if (ctr->halt) return;
  const uint32_t n = min(ctr->n[which], cap);
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t key = kInvalidCell, w = 0;
    if (i < n) {
      w = a.w[i];
      if (w > 0) key = a.cell[i];
    }
    const uint32_t rank = bin_add(cellacc, key, w);
    mark_tile(tiles, key, (uint64_t)rank << 32);
    if (key != kInvalidCell) a.rank[i] = rank;
  }
}

// ---- photon transport (final algorithm, step 6) -------------------------------------
// Photons counted by the previous step's reactions leave their cell in at most n_new
// computational photons; each is emitted uniformly in the cell, isotropically, and
// travels an exponential distance whose mean is log-uniform in [l1, l2].  Absorbed
// photons make one electron of the photon's weight plus as many positive ions in the
// absorbing cell; photons leaving the domain are removed.  Geometry in double.  The
// grid stride runs over wavefront-uniform bases, so that every lane takes part in the
// reservation of its cell's photon slots.

template <typename T>
__global__ void __launch_bounds__(kBlock) k_photons(Bank a, Counters* ctr, int which,
                                                   unsigned long long* cellacc, uint32_t* tiles,
                                                   uint32_t* ngamma,
                                                   uint32_t* nplus, StepConst k, int n_new,
                                                   double l1, double l2) {
  if (ctr->halt) return;
  const double two_pi = 6.283185307179586476925286766559;
  const double lr = l2 / l1;
  uint64_t absorbed = 0, lost = 0;
  const int lane = lane_id();
  for (uint32_t c0 = blockIdx.x * blockDim.x; c0 < k.ncell; c0 += gridDim.x * blockDim.x) {
    const uint32_t c = c0 + threadIdx.x;
    const uint32_t ng = c < k.ncell ? ngamma[c] : 0u;
    const uint32_t M = ng < (uint32_t)n_new ? ng : (uint32_t)n_new;
    if (__ballot(M > 0) == 0ull) continue;  // no photons in this wavefront's cells
    if (ng) ngamma[c] = 0;
    // one atomic per wavefront reserves the slots of all its photons: cell lane L owns
    // slots [incl_L - M_L, incl_L) after the wavefront's base (incl: inclusive prefix
    // of M over the lanes); a photon that leaves the domain leaves its slot dead
    // (weight 0), which the scatter skips
    uint32_t incl = M;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(incl, d, 64);
      if (lane >= d) incl += y;
    }
    const uint32_t tot = __shfl(incl, 63, 64);
    uint32_t base = 0;
    if (lane == 63) base = atomicAdd(&ctr->n[which], tot);
    base = __shfl(base, 63, 64);
    const uint32_t cw = c0 + (threadIdx.x & ~63u);  // the wavefront's first cell
    // the wavefront's photons spread over its lanes: photon p (slot base + p) belongs to
    // the first lane L with incl_L > p
    for (uint32_t p0 = 0; p0 < tot; p0 += 64) {
      const uint32_t pp = p0 + (uint32_t)lane;
      int L = 0;
#pragma unroll
      for (int st = 32; st >= 1; st >>= 1) {
        const uint32_t v = __shfl(incl, L + st - 1, 64);
        if (v <= pp) L += st;
      }
      const uint32_t inclL = __shfl(incl, L, 64), ngL = __shfl(ng, L, 64);
      if (pp >= tot) continue;
      const uint32_t ML = ngL < (uint32_t)n_new ? ngL : (uint32_t)n_new;
      const uint32_t sidx = pp - (inclL - ML), cc = cw + (uint32_t)L;
      const uint32_t w = ngL / ML + (sidx == 0 ? ngL % ML : 0u);
      const double ci = (double)(cc % (uint32_t)k.nx), cj = (double)((cc / (uint32_t)k.nx) % (uint32_t)k.ny),
                   ck = (double)(cc / ((uint32_t)k.nx * (uint32_t)k.ny));
      const uint4 A = philox_block(cc, sidx, k.step, TAG_PHOTON, 0, k.key);
      const uint4 B = philox_block(cc, sidx, k.step, TAG_PHOTON, 1, k.key);
      const double cth = 2.0 * u_co(A.w) - 1.0;
      const double sth = sqrt(fmax(0.0, 1.0 - cth * cth));
      const double ph = two_pi * u_co(B.x);
      const double ell = l1 * pow(lr, u_co(B.y));
      const double rg = -ell * log(u_oc(B.z)) / k.dx;
      const double y[3] = {ci + u24(A.x) + rg * (sth * cos(ph)), cj + u24(A.y) + rg * (sth * sin(ph)),
                           ck + u24(A.z) + rg * cth};
      const bool in = y[0] >= 0.0 && y[0] < k.nx && y[1] >= 0.0 && y[1] < k.ny && y[2] >= 0.0 &&
                      y[2] < k.nz;
      const uint32_t q = base + pp;
      if (!in) {
        lost += w;
        if (q < k.cap) a.w[q] = 0u;
        continue;
      }
      const double f[3] = {floor(y[0]), floor(y[1]), floor(y[2])};
      const uint32_t cell =
          (uint32_t)f[0] + (uint32_t)k.nx * ((uint32_t)f[1] + (uint32_t)k.ny * (uint32_t)f[2]);
      if (q >= k.cap) { atomicOr(&ctr->overflow, 1u); continue; }
      put<T>(a, q, cell, to_off<T>(y[0] - f[0]), to_off<T>(y[1] - f[1]), to_off<T>(y[2] - f[2]), w,
             make_id(KIND_PHOTO, k.step, cc, sidx));
      const unsigned long long old = atomicAdd(&cellacc[cell], (1ull << 32) | (unsigned long long)w);
      mark_tile(tiles, cell, old);
      a.rank[q] = (uint32_t)(old >> 32);
      atomicAdd(&nplus[cell], w);
      absorbed += w;
    }
  }
  absorbed = wave_sum64(absorbed);
  lost = wave_sum64(lost);
  if (lane_id() == 0) {
    if (absorbed) atomicAdd(&ctr->ph_absorbed, (unsigned long long)absorbed);
    if (lost) atomicAdd(&ctr->ph_lost, (unsigned long long)lost);
  }
}

// ---- counting sort by cell ------------------------------------------------------------
// Per 2048-cell tile: particle and occupied-cell counts of flagged tiles (reduce), an
// exclusive scan of the tile counts in groups of 1024 tiles (mid) and of the group
// totals (top), then per cell the first bank slot (start, written for occupied cells
// only) and the ascending list of occupied cells (down).  Scratch layout (u32):
// tile counts [2 nb] | tile prefixes within the group [2 nb] | group prefixes [2 ng + 2].

constexpr int kScanPer = 8;                     // cells per thread (k_scan_down unpacks two uint4)
constexpr int kScanTile = kBlock * kScanPer;    // cells per tile (1 << kTileShift)
static_assert(kScanTile == (1 << kTileShift), "scan tile and tile flags disagree");
static_assert(kScanPer == 8, "k_scan_down reads a thread's counts as two uint4");
constexpr int kScanGroup = 1024;                // tiles per mid-level group

template <int NT>
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // sh: NT / 64 + 1 words
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < NT / 64; ++i) { const uint32_t t = sh[i]; sh[i] = acc; acc += t; }
    sh[NT / 64] = acc;
  }
  __syncthreads();
  const uint32_t r = sh[wid] + x - v;
  *total = sh[NT / 64];
  __syncthreads();
  return r;
}

// ncell_dev (may be null) holds a device-side cell count that overrides ncell: the
// ensemble scans only the cells its slots occupy, with a grid sized for its pool.
__device__ __forceinline__ uint32_t scan_cells(uint32_t ncell, const uint32_t* ncell_dev) {
  return ncell_dev ? *ncell_dev : ncell;
}
__device__ __forceinline__ uint32_t scan_tiles(uint32_t ncell) {
  return (ncell + kScanTile - 1) / kScanTile;
}

__global__ void __launch_bounds__(kBlock) k_scan_reduce(const unsigned long long* cellacc,
                                                       uint32_t ncell_arg,
                                                       const uint32_t* ncell_dev,
                                                       uint32_t* tiles, uint32_t* cnt) {
  __shared__ uint32_t sh[2][kBlock / 64 + 1];
  const uint32_t ncell = scan_cells(ncell_arg, ncell_dev);
  const uint32_t nb = scan_tiles(ncell);
  for (uint32_t t = blockIdx.x; t < nb; t += gridDim.x) {
    if (tiles[t] == 0) {  // no particle was binned into this tile
      if (threadIdx.x == 0) { cnt[2 * t] = 0u; cnt[2 * t + 1] = 0u; }
      continue;
    }
    // only the tile totals are needed here: cells read in coalesced order
    const uint32_t c0 = t * kScanTile + threadIdx.x;
    uint32_t n = 0, oc = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      const uint32_t c = c0 + j * kBlock;
      if (c < ncell) {
        const uint32_t k = (uint32_t)(cellacc[c] >> 32);
        n += k;
        oc += k ? 1u : 0u;
      }
    }
    uint32_t t0, t1;
    block_exclusive_scan<kBlock>(n, sh[0], &t0);
    block_exclusive_scan<kBlock>(oc, sh[1], &t1);
    if (threadIdx.x == 0) {
      cnt[2 * t] = t0;
      cnt[2 * t + 1] = t1;
      tiles[t] = 0;  // cleared for the next binning
    }
  }
}

__global__ void __launch_bounds__(kScanGroup) k_scan_mid(const uint32_t* cnt, uint32_t* pre,
                                                        uint32_t* grp, uint32_t ncell_arg,
                                                        const uint32_t* ncell_dev) {
  __shared__ uint32_t sh[2][kScanGroup / 64 + 1];
  const uint32_t nb = scan_tiles(scan_cells(ncell_arg, ncell_dev));
  const uint32_t ng = (nb + kScanGroup - 1) / kScanGroup;
  for (uint32_t g = blockIdx.x; g < ng; g += gridDim.x) {
    const uint32_t t = g * kScanGroup + threadIdx.x;
    const uint32_t v0 = t < nb ? cnt[2 * t] : 0u, v1 = t < nb ? cnt[2 * t + 1] : 0u;
    uint32_t s0, s1;
    const uint32_t e0 = block_exclusive_scan<kScanGroup>(v0, sh[0], &s0);
    const uint32_t e1 = block_exclusive_scan<kScanGroup>(v1, sh[1], &s1);
    if (t < nb) { pre[2 * t] = e0; pre[2 * t + 1] = e1; }
    if (threadIdx.x == 0) { grp[2 * g] = s0; grp[2 * g + 1] = s1; }
  }
}

__global__ void __launch_bounds__(kScanGroup) k_scan_top(uint32_t* grp, uint32_t ncell_arg,
                                                        const uint32_t* ncell_dev) {
  // exclusive scan of the ng <= 1024 group totals; grp[2 ng ..] = grand totals
  __shared__ uint32_t sh[2][kScanGroup / 64 + 1];
  const uint32_t nb = scan_tiles(scan_cells(ncell_arg, ncell_dev));
  const uint32_t ng = (nb + kScanGroup - 1) / kScanGroup;
  const uint32_t g = threadIdx.x;
  const uint32_t v0 = g < ng ? grp[2 * g] : 0u, v1 = g < ng ? grp[2 * g + 1] : 0u;
  uint32_t s0, s1;
  const uint32_t e0 = block_exclusive_scan<kScanGroup>(v0, sh[0], &s0);
  const uint32_t e1 = block_exclusive_scan<kScanGroup>(v1, sh[1], &s1);
  if (g < ng) { grp[2 * g] = e0; grp[2 * g + 1] = e1; }
  if (threadIdx.x == 0) { grp[2 * ng] = s0; grp[2 * ng + 1] = s1; }
}

__global__ void __launch_bounds__(kBlock) k_scan_down(const unsigned long long* cellacc,
                                                     uint32_t ncell_arg, const uint32_t* ncell_dev,
                                                     const uint32_t* cnt, const uint32_t* pre,
                                                     const uint32_t* grp, uint32_t* start,
                                                     uint32_t* occ, Counters* ctr, int dest) {
  if (ctr->halt) return;
  __shared__ uint32_t sh[2][kBlock / 64 + 1];
  __shared__ __align__(16) uint32_t tile_n[kScanTile];
  const uint32_t ncell = scan_cells(ncell_arg, ncell_dev);
  const uint32_t nb = scan_tiles(ncell);
  for (uint32_t t = blockIdx.x; t < nb; t += gridDim.x) {
    if (cnt[2 * t] == 0u) continue;  // empty tile: no start entries, no occupied cells
    // counts read in coalesced order through LDS; each thread then takes eight
    // consecutive cells (the scan follows cell order)
    const uint32_t tb = t * kScanTile;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      const uint32_t i = (uint32_t)j * kBlock + threadIdx.x;
      tile_n[i] = tb + i < ncell ? (uint32_t)(cellacc[tb + i] >> 32) : 0u;
    }
    __syncthreads();
    const uint32_t c0 = tb + threadIdx.x * kScanPer;
    uint32_t n[kScanPer];
    uint32_t k = 0, oc = 0;
    const uint4 a0 = *reinterpret_cast<const uint4*>(tile_n + threadIdx.x * kScanPer);
    const uint4 a1 = *reinterpret_cast<const uint4*>(tile_n + threadIdx.x * kScanPer + 4);
    n[0] = a0.x; n[1] = a0.y; n[2] = a0.z; n[3] = a0.w;
    n[4] = a1.x; n[5] = a1.y; n[6] = a1.z; n[7] = a1.w;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      k += n[j];
      oc += n[j] ? 1u : 0u;
    }
    const uint32_t g = t / kScanGroup;
    uint32_t t0, t1;
    uint32_t p0 = block_exclusive_scan<kBlock>(k, sh[0], &t0) + pre[2 * t] + grp[2 * g];
    uint32_t p1 = block_exclusive_scan<kBlock>(oc, sh[1], &t1) + pre[2 * t + 1] + grp[2 * g + 1];
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      if (n[j]) {
        start[c0 + j] = p0;
        occ[p1++] = c0 + j;
        p0 += n[j];
      }
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    const uint32_t ng = (nb + kScanGroup - 1) / kScanGroup;
    const uint32_t total = grp[2 * ng], tocc = grp[2 * ng + 1];
    start[ncell] = total;
    ctr->sorted = total;
    ctr->n_occ = tocc;
    ctr->n[dest] = total;
    ctr->n_work = 0;
    ctr->n_big = 0;
    ctr->n_heavy = 0;
    ctr->n_huge = 0;
    ctr->n_cfull = 0;
    ctr->n_cmerge = 0;
  }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_scatter(Bank a, Bank b, Counters* ctr, int which,
                                                   const uint32_t* start, uint32_t cap) {
  if (ctr->halt) return;
  const uint32_t n = min(ctr->n[which], cap);
  if (n <= 2u * gridDim.x * blockDim.x) {
    // at most two passes of the grid: one particle per thread and pass (0.22 ms at
    // 9.5e6 particles, against 0.24 ms in the paired form below)
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
      const uint32_t w = a.w[i];
      if (w == 0) continue;
      const uint32_t cell = a.cell[i];
      const uint32_t q = start[cell] + a.rank[i];
      put<T>(b, q, cell, as<T>(a.ox)[i], as<T>(a.oy)[i], as<T>(a.oz)[i], w, a.id[i]);
    }
    return;
  }
  // many passes: two particles per thread and pass, every load unconditional so that
  // both particles' loads are in flight together (2.60 against 3.06 ms at 6.9e7
  // particles); a dead slot (weight 0) or a second index past n reads slot 0 and cell 0
  // instead (one cached line for all such lanes) and stores nothing
  const uint32_t stride = gridDim.x * blockDim.x * 2u;
  for (uint32_t i0 = blockIdx.x * blockDim.x * 2u + threadIdx.x; i0 < n; i0 += stride) {
    const uint32_t i1 = i0 + blockDim.x;
    const uint32_t w0 = a.w[i0], w1 = i1 < n ? a.w[i1] : 0u;
    const uint32_t j0 = w0 ? i0 : 0u, j1 = w1 ? i1 : 0u;
    const uint32_t c0 = a.cell[j0], c1 = a.cell[j1];
    const uint32_t r0 = a.rank[j0], r1 = a.rank[j1];
    const T x0 = as<T>(a.ox)[j0], y0 = as<T>(a.oy)[j0], z0 = as<T>(a.oz)[j0];
    const T x1 = as<T>(a.ox)[j1], y1 = as<T>(a.oy)[j1], z1 = as<T>(a.oz)[j1];
    const uint64_t d0 = a.id[j0], d1 = a.id[j1];
    const uint32_t s0 = start[w0 ? c0 : 0u], s1 = start[w1 ? c1 : 0u];
    if (w0) put<T>(b, s0 + r0, c0, x0, y0, z0, w0, d0);
    if (w1) put<T>(b, s1 + r1, c1, x1, y1, z1, w1, d1);
  }
}

// ---- queries and reductions -----------------------------------------------------------

__global__ void k_ngp(Bank a, Counters* ctr, int which, uint32_t* out, uint32_t cap) {
  const uint32_t n = min(ctr->n[which], cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t w = a.w[i];
    if (w) atomicAdd(&out[a.cell[i]], w);
  }
}

__global__ void k_reduce_particles(Bank a, Counters* ctr, int which, unsigned long long* out,
                                   uint32_t cap) {
  const uint32_t n = min(ctr->n[which], cap);
  uint64_t cnt = 0, W = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    if (i < n) {
      const uint32_t w = a.w[i];
      cnt += w ? 1 : 0;
      W += w;
    }
  }
  cnt = wave_sum64(cnt);
  W = wave_sum64(W);
  if (lane_id() == 0) {
    atomicAdd(&out[0], (unsigned long long)cnt);
    atomicAdd(&out[1], (unsigned long long)W);
  }
}

__global__ void k_reduce_cells(const uint32_t* p, const uint32_t* m, uint32_t ncell,
                               unsigned long long* out) {
  uint64_t sp = 0, sm = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < ncell; base += gridDim.x * blockDim.x) {
    const uint32_t c = base + threadIdx.x;
    if (c < ncell) { sp += p[c]; sm += m[c]; }
  }
  sp = wave_sum64(sp);
  sm = wave_sum64(sm);
  if (lane_id() == 0) {
    atomicAdd(&out[0], (unsigned long long)sp);
    atomicAdd(&out[1], (unsigned long long)sm);
  }
}

__global__ void k_fires_dense(const uint32_t* occ, const uint32_t* occ_fires, const Counters* ctr,
                              uint32_t* out) {
  const uint32_t n = ctr->n_occ;
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const uint32_t c = occ[j];
    for (int r = 0; r < 3; ++r) out[3 * (size_t)c + r] = occ_fires[3 * (size_t)j + r];
  }
}

__global__ void k_philox_fill(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, Key key,
                              uint64_t n, uint4* out) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = philox(make_uint4(c0 + (uint32_t)i, c1, c2, c3), key);
}

}  // namespace

// ---- launchers ---------------------------------------------------------------------------

static inline bool fp64(const itokmc_ctx* ctx) { return ctx->d.precision == ITOKMC_FP64; }

hipError_t launch_seed_gaussian(itokmc_ctx* ctx, const itokmc_seed_desc* sd) {
  StepConst k = make_const(ctx, 0.0);
  const int g = grid_for(sd->n0);
  if (fp64(ctx))
    k_seed_gaussian<double><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, k,
                                                       sd->n0, sd->centre[0], sd->centre[1],
                                                       sd->centre[2], sd->sigma);
  else
    k_seed_gaussian<float><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, k,
                                                      sd->n0, sd->centre[0], sd->centre[1],
                                                      sd->centre[2], sd->sigma);
  return hipGetLastError();
}

hipError_t launch_seed_neutral(itokmc_ctx* ctx, const itokmc_seed_desc* sd) {
  StepConst k = make_const(ctx, 0.0);
  const int g = grid_for(ctx->ncell);
  if (fp64(ctx))
    k_seed_neutral<double><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, k,
                                                      ctx->nplus, ctx->d.n_new, sd->n_peak,
                                                      sd->centre[0], sd->centre[1], sd->centre[2],
                                                      sd->sigma);
  else
    k_seed_neutral<float><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, k,
                                                     ctx->nplus, ctx->d.n_new, sd->n_peak,
                                                     sd->centre[0], sd->centre[1], sd->centre[2],
                                                     sd->sigma);
  return hipGetLastError();
}

static int particle_grid(const itokmc_ctx* ctx) {
  // persistent-style grid: enough blocks to fill 256 CUs several times over
  return grid_for(ctx->cap, kBlock, 4096);
}

hipError_t launch_push_uniform(itokmc_ctx* ctx, const StepConst& k) {
  const int g = particle_grid(ctx);
  if (fp64(ctx))
    k_push_uniform<double><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur,
                                                      ctx->cellacc, ctx->tiles, k);
  else
    k_push_uniform<float><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur,
                                                     ctx->cellacc, ctx->tiles, k);
  return hipGetLastError();
}

hipError_t launch_count(itokmc_ctx* ctx) {
  k_count<<<particle_grid(ctx), kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur,
                                                     ctx->cellacc, ctx->tiles, (uint32_t)ctx->cap);
  return hipGetLastError();
}

hipError_t launch_photons(itokmc_ctx* ctx, const StepConst& k) {
  if (!(ctx->c.kgamma_ratio > 0.0)) return hipSuccess;
  // up to 4096 workgroups: 0.149 ms per step at 9.5e6 particles against 0.21 ms with
  // 16384 and 0.17 ms with 2048
  const int g = grid_for(ctx->ncell, kBlock, 4096);
  if (fp64(ctx))
    k_photons<double><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur,
                                                 ctx->cellacc, ctx->tiles, ctx->ngamma, ctx->nplus, k,
                                                 ctx->d.n_new, ctx->c.photon_l1, ctx->c.photon_l2);
  else
    k_photons<float><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur,
                                                ctx->cellacc, ctx->tiles, ctx->ngamma, ctx->nplus, k,
                                                ctx->d.n_new, ctx->c.photon_l1, ctx->c.photon_l2);
  return hipGetLastError();
}

size_t scan_scratch_words(uint64_t ncell) {
  const uint64_t nb = (ncell + kScanTile - 1) / kScanTile + 1;
  const uint64_t ng = (nb + kScanGroup - 1) / kScanGroup + 1;
  return (size_t)(4 * nb + 2 * ng + 2);
}

hipError_t launch_scan_raw(const unsigned long long* cellacc, uint32_t max_cells,
                           const uint32_t* ncell_dev, uint32_t* tiles, uint32_t* scratch,
                           uint32_t* start, uint32_t* occ, Counters* ctr, int dest, hipStream_t s) {
  const uint32_t nb = (max_cells + kScanTile - 1) / kScanTile;
  uint32_t* cnt = scratch;
  uint32_t* pre = scratch + 2 * (size_t)(nb + 1);
  uint32_t* grp = scratch + 4 * (size_t)(nb + 1);
  const uint32_t gt = std::max<uint32_t>(1, std::min<uint32_t>(nb, 8192));  // tiles are looped over
  const uint32_t ng = std::max<uint32_t>(1, (nb + kScanGroup - 1) / kScanGroup);
  k_scan_reduce<<<gt, kBlock, 0, s>>>(cellacc, max_cells, ncell_dev, tiles, cnt);
  k_scan_mid<<<std::min<uint32_t>(ng, 1024), kScanGroup, 0, s>>>(cnt, pre, grp, max_cells, ncell_dev);
  k_scan_top<<<1, kScanGroup, 0, s>>>(grp, max_cells, ncell_dev);
  k_scan_down<<<gt, kBlock, 0, s>>>(cellacc, max_cells, ncell_dev, cnt, pre, grp, start, occ, ctr, dest);
  return hipGetLastError();
}

hipError_t launch_scan(itokmc_ctx* ctx) {
  return launch_scan_raw(ctx->cellacc, ctx->ncell, nullptr, ctx->tiles, ctx->blocksums, ctx->start,
                         ctx->occ, ctx->ctr, 1 - ctx->cur, ctx->s);
}

hipError_t launch_scatter_raw(Bank a, Bank b, Counters* ctr, int which, const uint32_t* start,
                              uint32_t cap, int fp64, int grid, hipStream_t s) {
  if (fp64)
    k_scatter<double><<<grid, kBlock, 0, s>>>(a, b, ctr, which, start, cap);
  else
    k_scatter<float><<<grid, kBlock, 0, s>>>(a, b, ctr, which, start, cap);
  return hipGetLastError();
}

hipError_t launch_scatter(itokmc_ctx* ctx) {
  // more workgroups than the other particle kernels: measured 0.197 ms at 9.5e6
  // particles with up to 32768 against 0.224 ms with 4096 (and 0.21 ms with 16384 or
  // 65536)
  const int g = grid_for(ctx->cap, kBlock, 32768);
  if (fp64(ctx))
    k_scatter<double><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->bank[1 - ctx->cur],
                                                 ctx->ctr, ctx->cur, ctx->start, (uint32_t)ctx->cap);
  else
    k_scatter<float><<<g, kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->bank[1 - ctx->cur],
                                                ctx->ctr, ctx->cur, ctx->start, (uint32_t)ctx->cap);
  return hipGetLastError();
}

hipError_t launch_ngp(itokmc_ctx* ctx, uint32_t* out) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(uint32_t) * ctx->ncell, ctx->s);
  if (e != hipSuccess) return e;
  k_ngp<<<particle_grid(ctx), kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, out,
                                                   (uint32_t)ctx->cap);
  return hipGetLastError();
}

hipError_t launch_reduce_particles(itokmc_ctx* ctx, unsigned long long* out2) {
  k_reduce_particles<<<particle_grid(ctx), kBlock, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr,
                                                                ctx->cur, out2, (uint32_t)ctx->cap);
  return hipGetLastError();
}

hipError_t launch_reduce_cells(itokmc_ctx* ctx, unsigned long long* out2) {
  k_reduce_cells<<<grid_for(ctx->ncell, kBlock, 4096), kBlock, 0, ctx->s>>>(
      ctx->nplus, ctx->nminus, ctx->ncell, out2);
  return hipGetLastError();
}

hipError_t launch_fires_dense(itokmc_ctx* ctx, uint32_t* out) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(uint32_t) * 3 * (size_t)ctx->ncell, ctx->s);
  if (e != hipSuccess) return e;
  k_fires_dense<<<grid_for(ctx->ncell, kBlock, 4096), kBlock, 0, ctx->s>>>(ctx->occ, ctx->occ_fires,
                                                                           ctx->ctr, out);
  return hipGetLastError();
}

hipError_t launch_philox_fill(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                              uint32_t k1, uint64_t n, uint32_t* out, hipStream_t s) {
  k_philox_fill<<<grid_for(n, kBlock, 4096), kBlock, 0, s>>>(c0, c1, c2, c3, Key{k0, k1}, n,
                                                             reinterpret_cast<uint4*>(out));
  return hipGetLastError();
}

}  // namespace itk
