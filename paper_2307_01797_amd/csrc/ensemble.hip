// Batched ensemble: many independent uniform-field realizations advanced together.
//
// Every realization (slot) owns 4096-cell blocks of a shared cell pool and a quota of a
// shared particle pool.  A global cell g belongs to block g >> 12; the block table gives
// its slot and its local block, and the slot's block map gives the global block of each
// local block, so a particle's global cell and its realization's own cell index convert
// both ways in O(1).  One ensemble step is the single-context step over the whole pool:
//   push + NGP binning (each particle with its slot's constants) -> counting sort over
//   the occupied pool cells -> scatter -> per-cell KMC (slot's rates, dt, key, step)
//   -> coupling of eq. w -> per-slot bookkeeping (step counter, stop rule).
// Ids, random streams and product positions use the local cell and the slot's own key,
// so each realization evolves exactly as it would alone.  The fixed kernel sequence is
// replayed as one HIP graph per bank parity.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "couple_device.hpp"
#include "device.hpp"
#include "itk.hpp"
#include "kmc_device.hpp"
#include "push_device.hpp"

namespace itk {
namespace {

constexpr int kBlkShift = 12;
constexpr uint32_t kBlkCells = 1u << kBlkShift;
constexpr uint32_t kBlkMask = kBlkCells - 1u;
constexpr int kMaxSlots = 4096;
constexpr int kListMax = 768;  // blocks per table-update launch (kernel argument space)
constexpr int kCUs = 256;

// Per-slot constants, written at admission; step and state advance on the device.
struct SlotConst {
  int nx, ny, nz;
  uint32_t ncell;
  Key key;
  uint32_t step, nsteps;
  uint32_t state, n_new, quota, map_off;
  uint64_t stop;
  KmcParams kp;
  double dt, diff;
  double drift[3];
  double k[3];
};

// Per-slot tallies, structure of arrays: st[f * max_slots + slot].
enum Stat {
  S_LIVE = 0,  // live particles pushed this step (reset each step)
  S_LEFT,      // of which left the grid (reset each step)
  S_PROD,      // product slots reserved this step (reset each step)
  S_CAPPED,    // quota overflow flag
  S_OUTW,      // cumulative outflow weight
  S_CREATED,   // cumulative computational particles created by the coupling
  S_REMOVED,   // cumulative weight removed by the coupling
  S_F0, S_F1, S_F2,
  S_PUSHED,    // cumulative particle-steps
  S_NUM
};

struct BlkList {
  uint32_t n, first_local;
  uint32_t b[kListMax];
};

template <typename T>
__device__ __forceinline__ T* as(void* p) { return reinterpret_cast<T*>(p); }

__device__ __forceinline__ uint32_t to_local(uint32_t g, const uint32_t* blk_local) {
  return (blk_local[g >> kBlkShift] << kBlkShift) | (g & kBlkMask);
}
__device__ __forceinline__ uint32_t to_global(uint32_t c, const uint32_t* map, uint32_t map_off) {
  return (map[map_off + (c >> kBlkShift)] << kBlkShift) | (c & kBlkMask);
}

// Segmented sum over runs of equal keys in the wavefront (inactive lanes: kInvalidCell);
// true in the last lane of each active run, with *total the run's sum.
__device__ __forceinline__ bool run_total(uint32_t key, uint64_t val, uint64_t* total) {
  const int lane = lane_id();
  const bool active = key != kInvalidCell;
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool head = (lane == 0) || (prev != key);
  const uint64_t heads = __ballot(head);
  const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int seg_start = 63 - __clzll(heads & upto);
  const uint64_t after = heads & ~upto;
  const int seg_end = after ? (__ffsll((long long)after) - 2) : 63;
  uint64_t x = active ? val : 0ull;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint64_t y = shfl_up64(x, d);
    if (lane - d >= seg_start) x += y;
  }
  *total = x;
  return active && lane == seg_end;
}

// ---- slot table maintenance (arguments by value: no host staging) --------------------

__global__ void e_set_slot(SlotConst v, int s, SlotConst* sc, unsigned long long* st,
                           uint32_t* stat2, uint32_t ms) {
  if (threadIdx.x == 0) {
    sc[s] = v;
    stat2[2 * s] = v.state;
    stat2[2 * s + 1] = 0;
  }
  if (threadIdx.x < S_NUM) st[threadIdx.x * ms + s] = 0ull;
}

__global__ void e_set_blocks(BlkList L, int s, uint32_t map_off, int32_t* blk_slot,
                             uint32_t* blk_local, uint32_t* map) {
  for (uint32_t i = threadIdx.x; i < L.n; i += blockDim.x) {
    const uint32_t b = L.b[i], lb = L.first_local + i;
    blk_slot[b] = s;
    blk_local[b] = lb;
    map[map_off + lb] = b;
  }
}

__global__ void e_clear_blocks(BlkList L, int s, SlotConst* sc, uint32_t* stat2,
                               int32_t* blk_slot) {
  for (uint32_t i = threadIdx.x; i < L.n; i += blockDim.x) blk_slot[L.b[i]] = -1;
  if (threadIdx.x == 0 && s >= 0) {
    sc[s].state = ITOKMC_SLOT_FREE;
    stat2[2 * s] = ITOKMC_SLOT_FREE;
  }
}

// Zero the ion counts of a slot's blocks (one workgroup per block).
__global__ void e_zero_cells(BlkList L, uint32_t* nplus, uint32_t* nminus) {
  const uint32_t b = L.b[blockIdx.x];
  for (uint32_t i = threadIdx.x; i < kBlkCells; i += blockDim.x) {
    nplus[(b << kBlkShift) + i] = 0u;
    nminus[(b << kBlkShift) + i] = 0u;
  }
}

__global__ void e_set_u32(uint32_t* p, uint32_t v) { *p = v; }

// ---- seeding ----------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) e_seed_gaussian(Bank b, Counters* ctr, int which,
                                                      const SlotConst* sc, int s,
                                                      const uint32_t* map, uint32_t cap,
                                                      uint64_t n0, double dx, double cx,
                                                      double cy, double cz, double sigma) {
  const SlotConst S = sc[s];
  const int lim[3] = {S.nx, S.ny, S.nz};
  const double c[3] = {cx, cy, cz};
  for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x; base < n0;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = base + threadIdx.x;
    bool keep = false;
    double xi[3];
    if (i < n0) keep = gaussian_seed_point(i, S.key, dx, lim, c, sigma, xi);
    const uint32_t q = wave_append(&ctr->n[which], keep ? 1u : 0u);
    if (keep) {
      if (q >= cap) {
        atomicOr(&ctr->overflow, 1u);
      } else {
        const double f[3] = {floor(xi[0]), floor(xi[1]), floor(xi[2])};
        const uint32_t lc =
            (uint32_t)f[0] + (uint32_t)S.nx * ((uint32_t)f[1] + (uint32_t)S.ny * (uint32_t)f[2]);
        b.cell[q] = to_global(lc, map, S.map_off);
        as<T>(b.ox)[q] = to_off<T>(xi[0] - f[0]);
        as<T>(b.oy)[q] = to_off<T>(xi[1] - f[1]);
        as<T>(b.oz)[q] = to_off<T>(xi[2] - f[2]);
        b.w[q] = 1u;
        b.id[q] = (1ull << 61) | i;
      }
    }
  }
}

// ---- the step ---------------------------------------------------------------------------

// Push with fused NGP binning over the pool.  Particles of released slots are dropped,
// particles of finished slots stay binned where they are.  A workgroup takes one
// contiguous chunk of the bank (whose particles mostly share a realization), and each
// thread keeps its realization's tallies in registers, flushing them when it moves to
// another realization and, wave-aggregated, at the end.
// bid, nblk: this workgroup's index and the number of workgroups taking part.
template <typename T>
__device__ __forceinline__ void push_phase(Bank a, Counters* ctr, int which,
                                           unsigned long long* cellacc, uint32_t* tiles,
                                           const SlotConst* sc, const int32_t* blk_slot,
                                           const uint32_t* blk_local, const uint32_t* map,
                                           unsigned long long* st, uint32_t ms, uint32_t cap,
                                           uint32_t bid, uint32_t nblk) {
  const uint32_t n = min(ctr->n[which], cap);
  const uint32_t per = ((n + nblk - 1) / nblk + blockDim.x - 1) / blockDim.x * blockDim.x;
  const uint32_t b0 = bid * per, b1 = min(n, b0 + per);
  uint32_t cur = kInvalidCell;
  uint64_t live = 0, left = 0, outw = 0;
  for (uint32_t base = b0; base < b1; base += blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t key = kInvalidCell, w = 0;
    // two rounds of loads instead of a chain: the particle's words (kept ahead of the
    // weight test by the empty asm), then its block's slot and local block
    uint32_t g = 0;
    T o0[3] = {(T)0, (T)0, (T)0};
    uint64_t id0 = 0;
    if (i < b1) {
      w = a.w[i];
      g = a.cell[i];
      o0[0] = as<T>(a.ox)[i];
      o0[1] = as<T>(a.oy)[i];
      o0[2] = as<T>(a.oz)[i];
      id0 = a.id[i];
    }
    asm volatile("" ::"v"(w), "v"(g), "v"(o0[0]), "v"(o0[1]), "v"(o0[2]), "v"(id0));
    if (w > 0) {
      const int s = blk_slot[g >> kBlkShift];
      const uint32_t lblk = blk_local[g >> kBlkShift];
      asm volatile("" ::"v"(s), "v"(lblk));
      if (s < 0) {
        a.w[i] = 0;  // realization released
      } else if (sc[s].state != ITOKMC_SLOT_ACTIVE) {
        key = g;
      } else {
        const SlotConst& S = sc[s];
        if ((uint32_t)s != cur) {
          if (cur != kInvalidCell) {
            if (live) atomicAdd(&st[S_LIVE * ms + cur], (unsigned long long)live);
            if (left) atomicAdd(&st[S_LEFT * ms + cur], (unsigned long long)left);
            if (outw) atomicAdd(&st[S_OUTW * ms + cur], (unsigned long long)outw);
          }
          cur = (uint32_t)s;
          live = left = outw = 0;
        }
        const uint32_t c = (lblk << kBlkShift) | (g & kBlkMask);  // the local cell index
        T o[3] = {o0[0], o0[1], o0[2]};
        int ci[3] = {(int)(c % (uint32_t)S.nx), (int)((c / (uint32_t)S.nx) % (uint32_t)S.ny),
                     (int)(c / ((uint32_t)S.nx * (uint32_t)S.ny))};
        const int lim[3] = {S.nx, S.ny, S.nz};
        const T drift[3] = {(T)S.drift[0], (T)S.drift[1], (T)S.drift[2]};
        const bool inside = push_uniform<T>(id0, S.step, S.key, drift, (T)S.diff, lim, ci, o);
        ++live;
        if (inside) {
          const uint32_t lc =
              (uint32_t)ci[0] + (uint32_t)S.nx * ((uint32_t)ci[1] + (uint32_t)S.ny * (uint32_t)ci[2]);
          key = to_global(lc, map, S.map_off);
          a.cell[i] = key;
          as<T>(a.ox)[i] = o[0];
          as<T>(a.oy)[i] = o[1];
          as<T>(a.oz)[i] = o[2];
        } else {
          a.w[i] = 0;
          ++left;
          outw += w;
        }
      }
    }
    const uint32_t rank = bin_add(cellacc, key, w);
    mark_tile(tiles, key, (uint64_t)rank << 32);
    if (key != kInvalidCell) a.rank[i] = rank;
  }
  uint64_t tot;
  if (run_total(cur, live, &tot) && tot) atomicAdd(&st[S_LIVE * ms + cur], (unsigned long long)tot);
  if (run_total(cur, left, &tot) && tot) atomicAdd(&st[S_LEFT * ms + cur], (unsigned long long)tot);
  if (run_total(cur, outw, &tot) && tot) atomicAdd(&st[S_OUTW * ms + cur], (unsigned long long)tot);
}

template <typename T>
__global__ void __launch_bounds__(1024) e_push(Bank a, Counters* ctr, int which,
                                              unsigned long long* cellacc, uint32_t* tiles,
                                              const SlotConst* sc,
                                              const int32_t* blk_slot, const uint32_t* blk_local,
                                              const uint32_t* map, unsigned long long* st,
                                              uint32_t ms, uint32_t cap) {
  push_phase<T>(a, ctr, which, cellacc, tiles, sc, blk_slot, blk_local, map, st, ms, cap,
                blockIdx.x, gridDim.x);
}

// Per-slot tallies of one thread, flushed to the slot's counters when the thread moves
// to another slot and, wave-aggregated, at the end.
struct SlotTally {
  uint32_t slot = kInvalidCell;
  uint64_t v[5] = {0, 0, 0, 0, 0};  // fires x3, created, removed weight
  static constexpr int kField[5] = {S_F0, S_F1, S_F2, S_CREATED, S_REMOVED};
  __device__ void flush(unsigned long long* st, uint32_t ms) {
    if (slot != kInvalidCell)
      for (int i = 0; i < 5; ++i)
        if (v[i]) atomicAdd(&st[kField[i] * ms + slot], (unsigned long long)v[i]);
    for (int i = 0; i < 5; ++i) v[i] = 0;
  }
  __device__ void add(uint32_t s, const uint64_t x[5], unsigned long long* st, uint32_t ms) {
    if (s != slot) { flush(st, ms); slot = s; }
    for (int i = 0; i < 5; ++i) v[i] += x[i];
  }
  // all lanes call: one atomic per run of equal slots in the wavefront
  __device__ void flush_wave(unsigned long long* st, uint32_t ms) {
    for (int i = 0; i < 5; ++i) {
      uint64_t tot;
      if (run_total(slot, v[i], &tot) && tot) atomicAdd(&st[kField[i] * ms + slot], (unsigned long long)tot);
      v[i] = 0;
    }
  }
};

// Per-cell KMC over the occupied pool cells; reserves product slots within each
// realization's quota and queues cells for the coupling.  As in the single-context
// step, a fast pass settles cells whose step is one SSA excursion and queues the rest,
// untouched, for the full pass; a thread takes kEnsKmcPer cells between the
// workgroup-aggregated appends.
constexpr int kEnsKmcPer = 4;

// sh: 18 words of LDS (block_append).
template <bool kFast>
__device__ __forceinline__ void kmc_phase(
    Counters* ctr, const uint32_t* occ, unsigned long long* cellacc, uint32_t* nplus,
    uint32_t* nminus, int32_t* dN, uint32_t* work, uint32_t* cbase, uint32_t* heavy,
    const SlotConst* sc, const int32_t* blk_slot, const uint32_t* blk_local,
    unsigned long long* st, uint32_t ms, int dest, uint32_t* sh, uint32_t bid, uint32_t nblk) {
  const uint32_t n = kFast ? ctr->n_occ : ctr->n_heavy;
  const uint32_t span = blockDim.x * kEnsKmcPer;
  SlotTally tally;
  for (uint32_t base = bid * span; base < n; base += nblk * span) {
    uint32_t js[kEnsKmcPer], Ms[kEnsKmcPer], fl[kEnsKmcPer];  // fl: 1 queue, 2 defer
    uint32_t nq = 0, nd = 0, nm = 0;
#pragma unroll
    for (int r = 0; r < kEnsKmcPer; ++r) {
      const uint32_t jj = base + (uint32_t)r * blockDim.x + threadIdx.x;
      js[r] = 0; Ms[r] = 0; fl[r] = 0;
      uint32_t skey = kInvalidCell, M = 0, j = 0, g = 0;
      int64_t d = 0;
      int64_t f[3] = {0, 0, 0};
      State X{0, 0, 0, 0};
      bool defer = false;
      if (jj < n) {
        j = kFast ? jj : heavy[jj];
        g = occ[j];
        const uint32_t Xe = (uint32_t)cellacc[g];
        const int s = blk_slot[g >> kBlkShift];
        if (s >= 0 && sc[s].state == ITOKMC_SLOT_ACTIVE) {
          const SlotConst& S = sc[s];
          const uint32_t c = to_local(g, blk_local);
          X = State{(int64_t)Xe, (int64_t)nplus[g], (int64_t)nminus[g], 0};
          const double k[3] = {S.k[0], S.k[1], S.k[2]};
          CellStream cs;
          cs.init(c, S.step, TAG_KMC, 0, S.key);
          if (kFast) defer = !advance_fast(S.kp, X, k, S.dt, cs, f);
          else advance(S.kp, X, k, S.dt, cs, f);
          if (!defer) {
            skey = (uint32_t)s;
            d = X.e - (int64_t)Xe;
            if (d > 0) M = d < (int64_t)S.n_new ? (uint32_t)d : S.n_new;
          }
        }
        if (!defer) cellacc[g] = 0ull;
      }
      // quota: live particles kept by the push plus products reserved so far
      const uint64_t before = run_add(st + S_PROD * ms, M ? skey : kInvalidCell, M);
      bool apply = skey != kInvalidCell;
      if (M) {
        const uint64_t kept = st[S_LIVE * ms + skey] - st[S_LEFT * ms + skey];
        if (kept + before + M > (uint64_t)sc[skey].quota) {
          // products dropped: the realization is capped and stops after this step.  The
          // cell keeps its state from before the reactions (ions, electrons and tallies
          // together), so that the realization's charge stays exact.
          M = 0;
          d = 0;
          f[0] = f[1] = f[2] = 0;
          apply = false;
          atomicOr(&st[S_CAPPED * ms + skey], 1ull);
        }
      }
      if (apply) {
        nplus[g] = (uint32_t)X.p;
        nminus[g] = (uint32_t)X.m;
      }
      if (jj < n && !defer) {
        dN[j] = (int32_t)d;
        js[r] = j;
        if (d != 0) { fl[r] = 1; ++nq; }
        Ms[r] = M;
        nm += M;
        if (skey != kInvalidCell) {
          const uint64_t x[5] = {(uint64_t)f[0], (uint64_t)f[1], (uint64_t)f[2], (uint64_t)M,
                                 d < 0 ? (uint64_t)(-d) : 0ull};
          tally.add(skey, x, st, ms);
        }
      } else if (defer) {
        js[r] = j; fl[r] = 2; ++nd;
      }
    }
    uint32_t hb = kFast ? block_append(&ctr->n_heavy, nd, sh) : 0u;
    uint32_t qb = block_append(&ctr->n_work, nq, sh);
    uint32_t mb = block_append(&ctr->n[dest], nm, sh);
#pragma unroll
    for (int r = 0; r < kEnsKmcPer; ++r) {
      if (fl[r] == 2) heavy[hb++] = js[r];
      if (fl[r] == 1) work[qb++] = js[r];
      if (Ms[r]) { cbase[js[r]] = mb; mb += Ms[r]; }
    }
  }
  tally.flush_wave(st, ms);
}

template <bool kFast>
__global__ void __launch_bounds__(kFast ? 256 : 64) e_kmc(
    Counters* ctr, const uint32_t* occ, unsigned long long* cellacc, uint32_t* nplus,
    uint32_t* nminus, int32_t* dN, uint32_t* work, uint32_t* cbase, uint32_t* heavy,
    const SlotConst* sc, const int32_t* blk_slot, const uint32_t* blk_local,
    unsigned long long* st, uint32_t ms, int dest) {
  __shared__ uint32_t sh[18];
  kmc_phase<kFast>(ctr, occ, cellacc, nplus, nminus, dN, work, cbase, heavy, sc, blk_slot,
                   blk_local, st, ms, dest, sh, blockIdx.x, gridDim.x);
}

// Coupling of eq. w, one wavefront per queued cell (no merge in the ensemble).
// wid, nwaves: this wavefront's index and the number of wavefronts taking part.
template <typename T>
__device__ __forceinline__ void couple_phase(Bank b, Counters* ctr, const uint32_t* work,
                                             const uint32_t* occ, const uint32_t* start,
                                             const int32_t* dN, const uint32_t* cbase,
                                             const SlotConst* sc, const int32_t* blk_slot,
                                             const uint32_t* blk_local, uint32_t cap, uint32_t wid,
                                             uint32_t nwaves) {
  const uint32_t nwork = ctr->n_work, n_occ = ctr->n_occ, sorted = ctr->sorted;
  const int lane = lane_id();
  for (uint32_t t = wid; t < nwork; t += nwaves) {
    const uint32_t j = work[t];
    const uint32_t g = occ[j];
    const int32_t d = dN[j];
    if (d < 0) {
      const uint32_t end = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
      (void)remove_weight(b, start[g], end, (uint32_t)(-d));
    }
    if (d > 0) {
      const int s = blk_slot[g >> kBlkShift];
      const SlotConst& S = sc[s];
      const uint32_t M = (uint32_t)d < S.n_new ? (uint32_t)d : S.n_new;
      const uint32_t wb = (uint32_t)d / M, wr = (uint32_t)d % M;
      if ((uint32_t)lane < M) {
        const uint32_t q = cbase[j] + (uint32_t)lane;
        if (q < cap)
          write_product<T>(b, q, g, to_local(g, blk_local), (uint32_t)lane, wb, wr, S.step, S.key);
        else
          atomicOr(&ctr->overflow, 1u);
      }
    }
  }
}

template <typename T>
__global__ void __launch_bounds__(64) e_couple(Bank b, Counters* ctr, const uint32_t* work,
                                              const uint32_t* occ, const uint32_t* start,
                                              const int32_t* dN, const uint32_t* cbase,
                                              const SlotConst* sc, const int32_t* blk_slot,
                                              const uint32_t* blk_local, uint32_t cap) {
  couple_phase<T>(b, ctr, work, occ, start, dN, cbase, sc, blk_slot, blk_local, cap, blockIdx.x,
                  gridDim.x);
}

// Per-slot end of step: advance the step counter and apply the stop rule (thread t of
// nthr threads takes slots t, t + nthr, ...).
__device__ __forceinline__ void finish_phase(SlotConst* sc, unsigned long long* st, uint32_t* stat2,
                                             uint32_t ms, uint32_t t, uint32_t nthr) {
  for (uint32_t s = t; s < ms; s += nthr) {
    if (sc[s].state != ITOKMC_SLOT_ACTIVE) continue;
    const uint64_t live = st[S_LIVE * ms + s];
    st[S_PUSHED * ms + s] += live;
    const uint32_t step = sc[s].step + 1u;
    sc[s].step = step;
    uint32_t state = ITOKMC_SLOT_ACTIVE;
    if (st[S_CAPPED * ms + s]) state = ITOKMC_SLOT_CAPPED;
    else if (step >= sc[s].nsteps || (sc[s].stop && live >= sc[s].stop)) state = ITOKMC_SLOT_DONE;
    sc[s].state = state;
    st[S_LIVE * ms + s] = 0ull;
    st[S_LEFT * ms + s] = 0ull;
    st[S_PROD * ms + s] = 0ull;
    stat2[2 * s] = state;
    stat2[2 * s + 1] = step;
  }
}

__global__ void e_finish(SlotConst* sc, unsigned long long* st, uint32_t* stat2, uint32_t ms) {
  finish_phase(sc, st, stat2, ms, blockIdx.x * blockDim.x + threadIdx.x, gridDim.x * blockDim.x);
}

// ---- persistent fused step ---------------------------------------------------------------
// The step above in one launch: a grid of kFuseBlock-thread workgroups that are all
// resident together (the host sizes it from the kernel's occupancy) runs every phase,
// with a device-wide barrier between consecutive phases.  A barrier waits a bounded
// time: a workgroup that gives up raises the grid's failure word and the overflow flag
// ITOKMC_OVF_BARRIER and returns, and the others return at their next wait once they see
// the word, so the launch always ends.  The counting sort takes a form suited to a
// resident grid: each workgroup counts one contiguous range of scan tiles, and after one
// barrier adds the totals of the ranges before its own to place its cells, so that the
// tile totals need no scan launches of their own.

constexpr int kFuseBlock = 256;
constexpr int kFuseMaxPerCu = 4;                          // register budgets: 1, 2 or 4 workgroups per CU
constexpr uint32_t kFuseMaxGrid = 1024u * kFuseMaxPerCu;  // workgroups (any compute-unit count up to 1024)
constexpr uint32_t kScanCells = 1u << kTileShift;         // cells per scan tile

// Barrier words, each on a 64-byte line of its own: one arrival count per group of
// workgroups (group g: the workgroups whose index is g modulo kBarGroups; the hardware
// deals consecutive workgroups to the eight XCDs in turn), the count of groups arrived,
// the number of barriers completed, and the failure word.
constexpr uint32_t kBarGroups = 8;
struct GridBar {
  uint32_t group[kBarGroups][16];
  uint32_t top[16];
  uint32_t gen[16];
  uint32_t fail[16];
};

// Device-wide barrier of the nblk workgroups of the grid; false once the grid has given
// up.  limit: the longest wait, in wall-clock ticks.  flag: one word of LDS.  A
// workgroup arrives at its group's count; the last of a group arrives at the top count,
// and the last group's arrival completes the barrier, so that no single word takes one
// atomic per workgroup.
__device__ bool grid_barrier(GridBar* bar, Counters* ctr, uint32_t nblk, uint64_t limit,
                             uint32_t* flag) {
  // every wavefront waits for its own stores of this phase to reach the L2; thread 0's
  // release fence then writes the L2's dirty lines back for the whole workgroup (the
  // workgroups of the grid sit on different XCDs, each with its own L2)
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    // the barrier words are read and counted with device-coherent relaxed atomics, so
    // the wait does not invalidate the caches that other workgroups are still using;
    // the acquire fence after the wait orders the reads of the next phase
    uint32_t ok = 1u;
    const uint32_t g = blockIdx.x % kBarGroups;
    const uint32_t ngroups = min(nblk, kBarGroups);
    const uint32_t gsize = (nblk - g + kBarGroups - 1u) / kBarGroups;  // workgroups of group g
    const uint32_t g0 = __hip_atomic_load(&bar->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    bool last = false;
    if (__hip_atomic_fetch_add(&bar->group[g][0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1u == gsize) {
      // the group's last arrival takes over the group's writes (acquire), resets the
      // group count and passes both on with its arrival at the top count (release)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      __hip_atomic_store(&bar->group[g][0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (__hip_atomic_fetch_add(&bar->top[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1u == ngroups) {
        __hip_atomic_store(&bar->top[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&bar->gen[0], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        last = true;
      }
    }
    if (!last) {
      const uint64_t t0 = wall_clock64();
      while (__hip_atomic_load(&bar->gen[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g0) {
        if (__hip_atomic_load(&bar->fail[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { ok = 0u; break; }
        if ((uint64_t)(wall_clock64() - t0) > limit) {
          __hip_atomic_fetch_or(&bar->fail[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicOr(&ctr->overflow, (uint32_t)ITOKMC_OVF_BARRIER);
          ok = 0u;
          break;
        }
        __builtin_amdgcn_s_sleep(1);
      }
    }
    *flag = ok;
  }
  __syncthreads();
  // every wavefront: its later reads see the other workgroups' writes of this phase
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  return *flag != 0u;
}

// Sums of two values over the workgroup (valid in every thread); sh: 2 * waves + 2 words.
__device__ __forceinline__ void block_sum2(uint32_t a, uint32_t b, uint32_t* sh, uint32_t* sa,
                                           uint32_t* sb) {
  const int lane = lane_id(), wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    a += (uint32_t)__shfl_xor((int)a, d, 64);
    b += (uint32_t)__shfl_xor((int)b, d, 64);
  }
  if (lane == 0) { sh[2 * wid] = a; sh[2 * wid + 1] = b; }
  __syncthreads();
  uint32_t x = 0, y = 0;
  for (int i = 0; i < nw; ++i) { x += sh[2 * i]; y += sh[2 * i + 1]; }
  *sa = x;
  *sb = y;
  __syncthreads();
}

// The scan tiles [t0, t1) of workgroup bid's range.
__device__ __forceinline__ void fuse_range(uint32_t ncell, uint32_t bid, uint32_t nblk,
                                           uint32_t* t0, uint32_t* t1) {
  const uint32_t nb = (ncell + kScanCells - 1) / kScanCells;
  const uint32_t per = (nb + nblk - 1) / nblk;
  *t0 = min(nb, bid * per);
  *t1 = min(nb, *t0 + per);
}

// Counting sort, first half: the particle and occupied-cell counts of every flagged
// tile of the range (flags cleared), and the range's totals in wgt[2 bid ..].
__device__ void fuse_count(const unsigned long long* cellacc, uint32_t ncell, uint32_t* tiles,
                           uint32_t* cnt, uint32_t* wgt, uint32_t* sh, uint32_t bid,
                           uint32_t nblk) {
  uint32_t t0, t1;
  fuse_range(ncell, bid, nblk, &t0, &t1);
  uint32_t tot0 = 0, tot1 = 0;
  for (uint32_t t = t0; t < t1; ++t) {
    uint32_t n = 0, oc = 0;
    if (tiles[t] != 0u) {  // uniform: one word per tile
      for (uint32_t c = t * kScanCells + threadIdx.x; c < min(ncell, (t + 1) * kScanCells); c += blockDim.x) {
        const uint32_t k = (uint32_t)(cellacc[c] >> 32);
        n += k;
        oc += k ? 1u : 0u;
      }
    }
    uint32_t sn, so;
    block_sum2(n, oc, sh, &sn, &so);
    if (threadIdx.x == 0) {
      cnt[2 * t] = sn;
      cnt[2 * t + 1] = so;
      tiles[t] = 0u;
    }
    tot0 += sn;
    tot1 += so;
  }
  if (threadIdx.x == 0) {
    wgt[2 * bid] = tot0;
    wgt[2 * bid + 1] = tot1;
  }
}

// Counting sort, second half: the first bank slot of every occupied cell of the range
// (start) and the ascending list of occupied cells (occ), offset by the totals of the
// ranges before this one; the last workgroup writes the grand totals and resets the
// step's append counters.  sh: kScanCells + 2 * waves + 2 words.
__device__ void fuse_place(const unsigned long long* cellacc, uint32_t ncell, const uint32_t* cnt,
                           const uint32_t* wgt, uint32_t* start, uint32_t* occ, Counters* ctr,
                           int dest, uint32_t* sh, uint32_t bid, uint32_t nblk) {
  uint32_t* red = sh + kScanCells;
  uint32_t b0 = 0, b1 = 0;
  for (uint32_t i = threadIdx.x; i < bid; i += blockDim.x) {
    b0 += wgt[2 * i];
    b1 += wgt[2 * i + 1];
  }
  uint32_t base0, base1;
  block_sum2(b0, b1, red, &base0, &base1);
  uint32_t t0, t1;
  fuse_range(ncell, bid, nblk, &t0, &t1);
  if (bid + 1u == nblk && threadIdx.x == 0) {
    const uint32_t total = base0 + wgt[2 * bid], tocc = base1 + wgt[2 * bid + 1];
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
  const uint32_t per = kScanCells / blockDim.x;  // consecutive cells per thread
  for (uint32_t t = t0; t < t1; ++t) {
    const uint32_t c0t = cnt[2 * t], c1t = cnt[2 * t + 1];
    if (c0t == 0u) continue;  // uniform
    const uint32_t tb = t * kScanCells;
    for (uint32_t i = threadIdx.x; i < kScanCells; i += blockDim.x)
      sh[i] = tb + i < ncell ? (uint32_t)(cellacc[tb + i] >> 32) : 0u;
    __syncthreads();
    uint32_t k = 0, oc = 0;
    for (uint32_t j = 0; j < per; ++j) {
      const uint32_t v = sh[threadIdx.x * per + j];
      k += v;
      oc += v ? 1u : 0u;
    }
    // exclusive prefix over the workgroup's threads, in cell order
    const int lane = lane_id(), wid = threadIdx.x >> 6, nw = (int)(blockDim.x >> 6);
    uint32_t x = k, y = oc;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t xs = (uint32_t)__shfl_up((int)x, d, 64), ys = (uint32_t)__shfl_up((int)y, d, 64);
      if (lane >= d) { x += xs; y += ys; }
    }
    if (lane == 63) { red[2 * wid] = x; red[2 * wid + 1] = y; }
    __syncthreads();
    uint32_t p0 = base0 + x - k, p1 = base1 + y - oc;
    for (int i = 0; i < wid; ++i) { p0 += red[2 * i]; p1 += red[2 * i + 1]; }
    for (uint32_t j = 0; j < per; ++j) {
      const uint32_t v = sh[threadIdx.x * per + j];
      if (v) {
        const uint32_t c = tb + threadIdx.x * per + j;
        start[c] = p0;
        occ[p1++] = c;
        p0 += v;
      }
    }
    __syncthreads();  // sh and red are reused by the next tile
    base0 += c0t;
    base1 += c1t;
    (void)nw;
  }
}

// Scatter into the destination bank at start[cell] + rank (thread t of nthr threads).
template <typename T>
__device__ __forceinline__ void fuse_scatter(Bank a, Bank b, const Counters* ctr, int which,
                                             const uint32_t* start, uint32_t cap, uint32_t t,
                                             uint32_t nthr) {
  const uint32_t n = min(ctr->n[which], cap);
  for (uint32_t i = t; i < n; i += nthr) {
    const uint32_t w = a.w[i];
    if (w == 0u) continue;
    const uint32_t cell = a.cell[i];
    const uint32_t q = start[cell] + a.rank[i];
    b.cell[q] = cell;
    as<T>(b.ox)[q] = as<T>(a.ox)[i];
    as<T>(b.oy)[q] = as<T>(a.oy)[i];
    as<T>(b.oz)[q] = as<T>(a.oz)[i];
    b.w[q] = w;
    b.id[q] = a.id[i];
  }
}

struct FuseArgs {
  Bank a, b;  // source and destination banks
  Counters* ctr;
  int cur;
  unsigned long long* cellacc;
  uint32_t* tiles;
  const uint32_t* ncell;  // pool cells to scan (device word)
  uint32_t *cnt, *wgt;
  GridBar* bar;
  uint32_t *start, *occ, *nplus, *nminus;
  int32_t* dN;
  uint32_t *work, *cbase, *heavy;
  SlotConst* sc;
  unsigned long long* st;
  uint32_t* stat2;
  const int32_t* blk_slot;
  const uint32_t *blk_local, *map;
  uint32_t ms, cap;
  uint64_t limit;
};

// W: resident workgroups per compute unit that the register budget is cut for (W waves
// per SIMD).  The full KMC pass needs about 256 registers per lane without spilling, so
// W = 1 keeps every phase in registers while W = 2 and 4 buy the push and the scatter
// more wavefronts in flight for spills in the KMC passes; the autotuner chooses.
template <typename T, int W>
__global__ void __launch_bounds__(kFuseBlock, W) e_step_fused(FuseArgs A) {
  __shared__ __align__(16) uint32_t sh[kScanCells + 2 * (kFuseBlock / 64) + 2];
  __shared__ uint32_t flag;
  const uint32_t bid = blockIdx.x, G = gridDim.x;
  const uint32_t tid = bid * blockDim.x + threadIdx.x, nthr = G * blockDim.x;
  const uint32_t nwv = blockDim.x >> 6;
  const int dest = 1 - A.cur;
  push_phase<T>(A.a, A.ctr, A.cur, A.cellacc, A.tiles, A.sc, A.blk_slot, A.blk_local, A.map, A.st,
                A.ms, A.cap, bid, G);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  const uint32_t ncell = *A.ncell;
  fuse_count(A.cellacc, ncell, A.tiles, A.cnt, A.wgt, sh, bid, G);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  fuse_place(A.cellacc, ncell, A.cnt, A.wgt, A.start, A.occ, A.ctr, dest, sh, bid, G);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  fuse_scatter<T>(A.a, A.b, A.ctr, A.cur, A.start, A.cap, tid, nthr);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  kmc_phase<true>(A.ctr, A.occ, A.cellacc, A.nplus, A.nminus, A.dN, A.work, A.cbase, A.heavy, A.sc,
                  A.blk_slot, A.blk_local, A.st, A.ms, dest, sh, bid, G);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  kmc_phase<false>(A.ctr, A.occ, A.cellacc, A.nplus, A.nminus, A.dN, A.work, A.cbase, A.heavy, A.sc,
                   A.blk_slot, A.blk_local, A.st, A.ms, dest, sh, bid, G);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  couple_phase<T>(A.b, A.ctr, A.work, A.occ, A.start, A.dN, A.cbase, A.sc, A.blk_slot, A.blk_local,
                  A.cap, bid * nwv + (threadIdx.x >> 6), G * nwv);
  if (!grid_barrier(A.bar, A.ctr, G, A.limit, &flag)) return;
  finish_phase(A.sc, A.st, A.stat2, A.ms, tid, nthr);
}

// ---- queries ------------------------------------------------------------------------------

template <typename T>
__global__ void __launch_bounds__(256) e_extract(Bank a, const Counters* ctr, int which,
                                                uint32_t cap, int s, const int32_t* blk_slot,
                                                const uint32_t* blk_local, Bank o,
                                                uint32_t* count) {
  const uint32_t n = min(ctr->n[which], cap);
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    bool mine = false;
    if (i < n && a.w[i] > 0) mine = blk_slot[a.cell[i] >> kBlkShift] == s;
    const uint32_t q = wave_append(count, mine ? 1u : 0u);
    if (mine) {
      o.cell[q] = to_local(a.cell[i], blk_local);
      as<T>(o.ox)[q] = as<T>(a.ox)[i];
      as<T>(o.oy)[q] = as<T>(a.oy)[i];
      as<T>(o.oz)[q] = as<T>(a.oz)[i];
      o.w[q] = a.w[i];
      o.id[q] = a.id[i];
    }
  }
}

// Live particle count and weight of every slot in one pool pass (out: 2 per slot).
__global__ void __launch_bounds__(256) e_reduce_all(Bank a, const Counters* ctr, int which,
                                                   uint32_t cap, const int32_t* blk_slot,
                                                   unsigned long long* out) {
  const uint32_t n = min(ctr->n[which], cap);
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t key = kInvalidCell, w = 0;
    if (i < n) {
      w = a.w[i];
      if (w > 0) {
        const int s = blk_slot[a.cell[i] >> kBlkShift];
        if (s >= 0) key = (uint32_t)s;
      }
    }
    uint64_t tot;
    if (run_total(key, 1ull, &tot)) atomicAdd(&out[2 * key], (unsigned long long)tot);
    if (run_total(key, (uint64_t)w, &tot)) atomicAdd(&out[2 * key + 1], (unsigned long long)tot);
  }
}

// Ion sums of the listed blocks into out[2 idx[i] ..] (one workgroup per block).
__global__ void __launch_bounds__(256) e_reduce_ions_multi(BlkList L, BlkList idx,
                                                          const uint32_t* nplus,
                                                          const uint32_t* nminus,
                                                          unsigned long long* out) {
  const uint32_t b = L.b[blockIdx.x], k = idx.b[blockIdx.x];
  uint64_t p = 0, m = 0;
  for (uint32_t i = threadIdx.x; i < kBlkCells; i += blockDim.x) {
    p += nplus[(b << kBlkShift) + i];
    m += nminus[(b << kBlkShift) + i];
  }
  p = wave_sum64(p);
  m = wave_sum64(m);
  if (lane_id() == 0) {
    if (p) atomicAdd(&out[2 * k], (unsigned long long)p);
    if (m) atomicAdd(&out[2 * k + 1], (unsigned long long)m);
  }
}

// First-fit allocator of contiguous index ranges (block-map entries).
struct RangeAlloc {
  std::map<uint32_t, uint32_t> free_;  // start -> length
  void init(uint32_t n) { free_.clear(); if (n) free_[0] = n; }
  bool take(uint32_t n, uint32_t* at) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *at = it->first;
        const uint32_t rest = it->second - n, st = it->first + n;
        free_.erase(it);
        if (rest) free_[st] = rest;
        return true;
      }
    }
    return false;
  }
  void give(uint32_t at, uint32_t n) {
    if (!n) return;
    auto it = free_.emplace(at, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct SlotHost {
  bool used = false, reported = false;
  std::vector<uint32_t> blocks;
  uint32_t map_off = 0;
  uint64_t quota = 0;
  itokmc_grid_desc d{};
  itokmc_coeffs c{};
  itokmc_run_desc r{};
};

}  // namespace
}  // namespace itk

using namespace itk;

struct itokmc_ens {
  itokmc_ens_desc d{};
  hipStream_t s = nullptr;
  char* arena = nullptr;
  uint32_t nblk = 0, ms = 0, max_cells = 0;
  uint32_t cap = 0;
  int cur = 0;
  Bank bank[2];
  unsigned long long* cellacc = nullptr;
  uint32_t *start = nullptr, *occ = nullptr, *nplus = nullptr, *nminus = nullptr;
  int32_t* dN = nullptr;
  uint32_t *work = nullptr, *cbase = nullptr, *blocksums = nullptr;
  Counters* ctr = nullptr;
  uint32_t* misc = nullptr;  // [0] cells to scan, [1] extraction counter
  unsigned long long* reduce = nullptr;
  SlotConst* sc = nullptr;
  unsigned long long* st = nullptr;
  uint32_t* stat2 = nullptr;
  int32_t* blk_slot = nullptr;
  uint32_t *blk_local = nullptr, *map = nullptr;
  unsigned long long* slot_red = nullptr;  // 4 per slot: count, weight (pool), n+, n-
  uint32_t* tiles = nullptr;                // scan tile flags
  uint32_t* heavy = nullptr;                // cells for the full KMC pass
  GridBar* bar = nullptr;                   // fused step: device-wide barrier words
  uint32_t* wgt = nullptr;                  // fused step: per-workgroup range totals
  int n_cu = 0;                             // compute units of the device
  int fuse_occ = 0;                         // fused kernel: resident workgroups per CU
  uint64_t fuse_limit = 0;                  // fused kernel: longest barrier wait (ticks)
  // host bookkeeping
  std::vector<SlotHost> slots;
  std::set<uint32_t> free_blocks, used_blocks;
  std::vector<uint32_t> pending_blocks;
  std::vector<std::pair<uint32_t, uint32_t>> pending_map;
  RangeAlloc map_alloc;
  uint64_t quota_free = 0, pending_quota = 0;
  uint32_t hw_blocks = 0;
  uint64_t steps = 0;
  itokmc_ens_tuning tune{256, 8, 256, 64, 1, 0};  // fused_per_cu 0: the kernel sequence
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool graph_failed = false;
  uint32_t* host_stat = nullptr;
  Counters* host_ctr = nullptr;
  unsigned long long* host_red = nullptr;
  std::string err;
};

namespace {

int ens_error(itokmc_ens* e, int code, const char* fmt, ...) {
  if (e) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    e->err = buf;
  }
  return code;
}

int ens_hip(itokmc_ens* e, hipError_t h, const char* what) {
  if (h == hipSuccess) return ITOKMC_OK;
  return ens_error(e, ITOKMC_EHIP, "%s: %s", what, hipGetErrorString(h));
}

size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

struct EnsLayout {
  size_t off[40];
  size_t total;
};

bool valid_ens(const itokmc_ens_desc* d) {
  if (!d) return false;
  if (d->max_slots < 1 || d->max_slots > kMaxSlots) return false;
  if (d->precision != ITOKMC_FP32 && d->precision != ITOKMC_FP64) return false;
  if (d->max_cells < 1 || d->max_cells > (1ull << 31)) return false;
  if (d->max_particles < 1 || d->max_particles > 0x7FFFFFFFull) return false;
  return true;
}

void ens_layout(const itokmc_ens_desc* d, EnsLayout* L) {
  const uint64_t nblk = (d->max_cells + kBlkCells - 1) / kBlkCells;
  const uint64_t nc = nblk * kBlkCells;
  const uint64_t cap = d->max_particles;
  const uint64_t ms = (uint64_t)d->max_slots;
  const size_t T = d->precision == ITOKMC_FP64 ? 8 : 4;
  size_t o = 0;
  int i = 0;
  auto put = [&](size_t bytes) { L->off[i++] = o; o += al(bytes); };
  for (int b = 0; b < 2; ++b) {
    put(cap * 4); put(cap * T); put(cap * T); put(cap * T); put(cap * 4); put(cap * 8); put(cap * 4);
  }
  put(nc * 8);                         // 14 cellacc
  put((nc + 1) * 4);                   // 15 start
  put(nc * 4);                         // 16 occ
  put(nc * 4);                         // 17 nplus
  put(nc * 4);                         // 18 nminus
  put(nc * 4);                         // 19 dN
  put(nc * 4);                         // 20 work
  put(nc * 4);                         // 21 cbase
  put(scan_scratch_words(nc) * 4);     // 22 scan scratch
  put(sizeof(Counters));               // 23 counters
  put(64);                             // 24 misc
  put(64);                             // 25 reduction scratch
  put(ms * sizeof(SlotConst));         // 26 slot constants
  put(ms * S_NUM * 8);                 // 27 tallies
  put(ms * 8);                         // 28 state and step
  put(nblk * 4);                       // 29 block -> slot
  put(nblk * 4);                       // 30 block -> local block
  put(2 * nblk * 4);                   // 31 block maps
  put(ms * 4 * 8);                     // 32 per-slot result reductions
  put((nc / 2048 + 2) * 4);            // 33 scan tile flags
  put(nc * 4);                         // 34 cells for the full KMC pass
  put(sizeof(GridBar) + 2 * kFuseMaxGrid * 4);  // 35 fused step: barrier words, range totals
  L->total = o;
}

inline bool f64(const itokmc_ens* e) { return e->d.precision == ITOKMC_FP64; }

int grid_particles(const itokmc_ens* e) {
  int g = kCUs * e->tune.push_blocks_per_cu;
  const uint64_t need = ((uint64_t)e->cap + e->tune.push_block - 1) / e->tune.push_block;
  if ((uint64_t)g > need) g = (int)std::max<uint64_t>(need, 1);
  return g;
}

template <typename T, int W>
hipError_t fuse_launch(const FuseArgs& A, uint32_t grid, hipStream_t s) {
  e_step_fused<T, W><<<grid, kFuseBlock, 0, s>>>(A);
  return hipGetLastError();
}

template <typename T>
hipError_t fuse_occupancy(int w, int* occ) {
  if (w == 1) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, e_step_fused<T, 1>, kFuseBlock, 0);
  if (w == 2) return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, e_step_fused<T, 2>, kFuseBlock, 0);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, e_step_fused<T, 4>, kFuseBlock, 0);
}

// The device's compute units, the fused budgets that keep their W workgroups per
// compute unit resident (a bit mask over W = 1, 2, 4) and the barrier time limit: 4 s of
// the device's constant-rate wall clock, or ITOKMC_FUSED_WAIT_US microseconds when that
// environment variable is set (tests shorten it to exercise the failure report).
hipError_t fuse_setup(itokmc_ens* e) {
  int dev = 0, rate_khz = 0;
  hipError_t h = hipGetDevice(&dev);
  if (h == hipSuccess) h = hipDeviceGetAttribute(&e->n_cu, hipDeviceAttributeMultiprocessorCount, dev);
  if (h == hipSuccess) h = hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev);
  e->fuse_occ = 0;
  for (int w : {1, 2, 4}) {
    int occ = 0;
    if (h == hipSuccess) h = f64(e) ? fuse_occupancy<double>(w, &occ) : fuse_occupancy<float>(w, &occ);
    if (h == hipSuccess && occ >= w) e->fuse_occ |= w;
  }
  if (h != hipSuccess) return h;
  if ((uint64_t)e->n_cu * kFuseMaxPerCu > kFuseMaxGrid) e->fuse_occ = 0;  // range totals would not fit
  uint64_t wait_us = 4000000ull;
  if (const char* v = getenv("ITOKMC_FUSED_WAIT_US")) wait_us = strtoull(v, nullptr, 10);
  e->fuse_limit = (uint64_t)std::max(rate_khz, 1) * wait_us / 1000ull;
  return hipSuccess;
}

hipError_t enqueue_fused(itokmc_ens* e, int cur, hipStream_t s) {
  FuseArgs A;
  A.a = e->bank[cur];
  A.b = e->bank[1 - cur];
  A.ctr = e->ctr;
  A.cur = cur;
  A.cellacc = e->cellacc;
  A.tiles = e->tiles;
  A.ncell = e->misc;
  A.cnt = e->blocksums;
  A.wgt = e->wgt;
  A.bar = e->bar;
  A.start = e->start;
  A.occ = e->occ;
  A.nplus = e->nplus;
  A.nminus = e->nminus;
  A.dN = e->dN;
  A.work = e->work;
  A.cbase = e->cbase;
  A.heavy = e->heavy;
  A.sc = e->sc;
  A.st = e->st;
  A.stat2 = e->stat2;
  A.blk_slot = e->blk_slot;
  A.blk_local = e->blk_local;
  A.map = e->map;
  A.ms = e->ms;
  A.cap = e->cap;
  A.limit = e->fuse_limit;
  const int w = e->tune.fused_per_cu;
  const uint32_t G = (uint32_t)(e->n_cu * w);  // exactly the resident workgroups
  if (f64(e))
    return w == 1 ? fuse_launch<double, 1>(A, G, s) : w == 2 ? fuse_launch<double, 2>(A, G, s)
                                                             : fuse_launch<double, 4>(A, G, s);
  return w == 1 ? fuse_launch<float, 1>(A, G, s) : w == 2 ? fuse_launch<float, 2>(A, G, s)
                                                          : fuse_launch<float, 4>(A, G, s);
}

// Enqueue one ensemble step for bank parity cur on stream s.
hipError_t enqueue_step(itokmc_ens* e, int cur, hipStream_t s) {
  if (e->tune.fused_per_cu > 0) return enqueue_fused(e, cur, s);
  const int dest = 1 - cur;
  const int gp = grid_particles(e);
  if (f64(e))
    e_push<double><<<gp, e->tune.push_block, 0, s>>>(e->bank[cur], e->ctr, cur, e->cellacc, e->tiles, e->sc,
                                                     e->blk_slot, e->blk_local, e->map, e->st, e->ms,
                                                     e->cap);
  else
    e_push<float><<<gp, e->tune.push_block, 0, s>>>(e->bank[cur], e->ctr, cur, e->cellacc, e->tiles, e->sc,
                                                    e->blk_slot, e->blk_local, e->map, e->st, e->ms,
                                                    e->cap);
  hipError_t h = hipGetLastError();
  if (h != hipSuccess) return h;
  h = launch_scan_raw(e->cellacc, e->max_cells, e->misc, e->tiles, e->blocksums, e->start, e->occ,
                      e->ctr, dest, s);
  if (h != hipSuccess) return h;
  h = launch_scatter_raw(e->bank[cur], e->bank[dest], e->ctr, cur, e->start, e->cap, f64(e) ? 1 : 0,
                         std::max(1, (int)std::min<uint64_t>((uint64_t)kCUs * 8, (e->cap + 255) / 256)), s);
  if (h != hipSuccess) return h;
  const uint64_t span = (uint64_t)e->tune.kmc_block * kEnsKmcPer;
  int gk = (int)std::min<uint64_t>((uint64_t)kCUs * 16, ((uint64_t)e->max_cells + span - 1) / span);
  if (gk < 1) gk = 1;
  e_kmc<true><<<gk, e->tune.kmc_block, 0, s>>>(e->ctr, e->occ, e->cellacc, e->nplus, e->nminus, e->dN,
                                               e->work, e->cbase, e->heavy, e->sc, e->blk_slot,
                                               e->blk_local, e->st, e->ms, dest);
  h = hipGetLastError();
  if (h != hipSuccess) return h;
  e_kmc<false><<<kCUs * 4, 64, 0, s>>>(e->ctr, e->occ, e->cellacc, e->nplus, e->nminus, e->dN, e->work,
                                       e->cbase, e->heavy, e->sc, e->blk_slot, e->blk_local, e->st,
                                       e->ms, dest);
  h = hipGetLastError();
  if (h != hipSuccess) return h;
  const int gc = kCUs * e->tune.couple_per_cu;
  if (f64(e))
    e_couple<double><<<gc, 64, 0, s>>>(e->bank[dest], e->ctr, e->work, e->occ, e->start, e->dN,
                                       e->cbase, e->sc, e->blk_slot, e->blk_local, e->cap);
  else
    e_couple<float><<<gc, 64, 0, s>>>(e->bank[dest], e->ctr, e->work, e->occ, e->start, e->dN,
                                      e->cbase, e->sc, e->blk_slot, e->blk_local, e->cap);
  h = hipGetLastError();
  if (h != hipSuccess) return h;
  e_finish<<<(e->ms + 255) / 256, 256, 0, s>>>(e->sc, e->st, e->stat2, e->ms);
  return hipGetLastError();
}

void drop_graphs(itokmc_ens* e) {
  for (int p = 0; p < 2; ++p)
    if (e->graph[p]) { (void)hipGraphExecDestroy(e->graph[p]); e->graph[p] = nullptr; }
  e->graph_failed = false;
}

bool capture_graphs(itokmc_ens* e) {
  if (e->graph[0] && e->graph[1]) return true;
  if (e->graph_failed) return false;
  for (int p = 0; p < 2; ++p) {
    if (e->graph[p]) continue;
    hipStream_t cs = nullptr;
    if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) { e->graph_failed = true; return false; }
    hipGraph_t g = nullptr;
    bool ok = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const hipError_t h = enqueue_step(e, p, cs);
      const bool end_ok = hipStreamEndCapture(cs, &g) == hipSuccess && g != nullptr;
      ok = h == hipSuccess && end_ok;
    }
    hipGraphExec_t ex = nullptr;
    if (ok) ok = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess;
    if (g) (void)hipGraphDestroy(g);
    (void)hipStreamDestroy(cs);
    (void)hipGetLastError();
    if (!ok) { drop_graphs(e); e->graph_failed = true; return false; }
    e->graph[p] = ex;
  }
  return true;
}

// Launch a block list in chunks of kListMax.
template <typename F>
hipError_t for_lists(const std::vector<uint32_t>& blocks, F f) {
  BlkList L;
  for (size_t i = 0; i < blocks.size(); i += kListMax) {
    L.n = (uint32_t)std::min<size_t>(kListMax, blocks.size() - i);
    L.first_local = (uint32_t)i;
    for (uint32_t k = 0; k < L.n; ++k) L.b[k] = blocks[i + k];
    hipError_t h = f(L);
    if (h != hipSuccess) return h;
  }
  return hipSuccess;
}

hipError_t update_hw(itokmc_ens* e) {
  const uint32_t hw = e->used_blocks.empty() ? 0u : *e->used_blocks.rbegin() + 1u;
  if (hw == e->hw_blocks) return hipSuccess;
  e->hw_blocks = hw;
  e_set_u32<<<1, 1, 0, e->s>>>(e->misc, hw * kBlkCells);
  return hipGetLastError();
}

int check_slot(itokmc_ens* e, int32_t slot) {
  if (!e) return ITOKMC_EINVAL;
  if (slot < 0 || slot >= (int32_t)e->ms || !e->slots[slot].used)
    return ens_error(e, ITOKMC_EINVAL, "slot %d is not in use", slot);
  return ITOKMC_OK;
}

}  // namespace

extern "C" {

size_t itokmc_ensemble_arena_bytes(const itokmc_ens_desc* desc) {
  if (!valid_ens(desc)) return 0;
  EnsLayout L;
  ens_layout(desc, &L);
  return L.total;
}

int itokmc_ensemble_create(itokmc_ens** out, const itokmc_ens_desc* desc, void* arena,
                           size_t arena_bytes, void* stream) {
  if (!out) return ITOKMC_EINVAL;
  *out = nullptr;
  if (!valid_ens(desc)) return ITOKMC_EINVAL;
  EnsLayout L;
  ens_layout(desc, &L);
  if (!arena || ((uintptr_t)arena & 255)) return ITOKMC_EINVAL;
  if (arena_bytes < L.total) return ITOKMC_ENOMEM;
  itokmc_ens* e = new itokmc_ens();
  e->d = *desc;
  e->s = (hipStream_t)stream;
  e->arena = (char*)arena;
  e->ms = (uint32_t)desc->max_slots;
  e->nblk = (uint32_t)((desc->max_cells + kBlkCells - 1) / kBlkCells);
  e->max_cells = e->nblk * kBlkCells;
  e->cap = (uint32_t)desc->max_particles;
  char* a = e->arena;
  for (int b = 0; b < 2; ++b) {
    Bank& k = e->bank[b];
    const int o = 7 * b;
    k.cell = (uint32_t*)(a + L.off[o]);
    k.ox = a + L.off[o + 1];
    k.oy = a + L.off[o + 2];
    k.oz = a + L.off[o + 3];
    k.w = (uint32_t*)(a + L.off[o + 4]);
    k.id = (uint64_t*)(a + L.off[o + 5]);
    k.rank = (uint32_t*)(a + L.off[o + 6]);
  }
  e->cellacc = (unsigned long long*)(a + L.off[14]);
  e->start = (uint32_t*)(a + L.off[15]);
  e->occ = (uint32_t*)(a + L.off[16]);
  e->nplus = (uint32_t*)(a + L.off[17]);
  e->nminus = (uint32_t*)(a + L.off[18]);
  e->dN = (int32_t*)(a + L.off[19]);
  e->work = (uint32_t*)(a + L.off[20]);
  e->cbase = (uint32_t*)(a + L.off[21]);
  e->blocksums = (uint32_t*)(a + L.off[22]);
  e->ctr = (Counters*)(a + L.off[23]);
  e->misc = (uint32_t*)(a + L.off[24]);
  e->reduce = (unsigned long long*)(a + L.off[25]);
  e->sc = (SlotConst*)(a + L.off[26]);
  e->st = (unsigned long long*)(a + L.off[27]);
  e->stat2 = (uint32_t*)(a + L.off[28]);
  e->blk_slot = (int32_t*)(a + L.off[29]);
  e->blk_local = (uint32_t*)(a + L.off[30]);
  e->map = (uint32_t*)(a + L.off[31]);
  e->slot_red = (unsigned long long*)(a + L.off[32]);
  e->tiles = (uint32_t*)(a + L.off[33]);
  e->heavy = (uint32_t*)(a + L.off[34]);
  e->bar = (GridBar*)(a + L.off[35]);
  e->wgt = (uint32_t*)(a + L.off[35] + sizeof(GridBar));
  hipError_t h = fuse_setup(e);
  if (h == hipSuccess) h = hipMemsetAsync(e->cellacc, 0, (size_t)e->max_cells * 8, e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->ctr, 0, sizeof(Counters), e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->misc, 0, 64, e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->tiles, 0, ((size_t)e->max_cells / 2048 + 2) * 4, e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->sc, 0, (size_t)e->ms * sizeof(SlotConst), e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->st, 0, (size_t)e->ms * S_NUM * 8, e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->stat2, 0, (size_t)e->ms * 8, e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->blk_slot, 0xFF, (size_t)e->nblk * 4, e->s);
  if (h == hipSuccess) h = hipMemsetAsync(e->bar, 0, sizeof(GridBar), e->s);
  if (h == hipSuccess) h = hipHostMalloc((void**)&e->host_stat, (size_t)e->ms * 8, hipHostMallocDefault);
  if (h == hipSuccess) h = hipHostMalloc((void**)&e->host_ctr, sizeof(Counters), hipHostMallocDefault);
  if (h == hipSuccess) h = hipHostMalloc((void**)&e->host_red, 64, hipHostMallocDefault);
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  if (h != hipSuccess) {
    if (e->host_stat) (void)hipHostFree(e->host_stat);
    if (e->host_ctr) (void)hipHostFree(e->host_ctr);
    if (e->host_red) (void)hipHostFree(e->host_red);
    delete e;
    return ITOKMC_EHIP;
  }
  e->slots.resize(e->ms);
  for (uint32_t b = 0; b < e->nblk; ++b) e->free_blocks.insert(b);
  e->map_alloc.init(2 * e->nblk);
  e->quota_free = e->cap;
  *out = e;
  return ITOKMC_OK;
}

int itokmc_ensemble_admit(itokmc_ens* e, const itokmc_grid_desc* d, const itokmc_coeffs* c,
                          const itokmc_seed_desc* sd, const itokmc_run_desc* r, int32_t* slot) {
  if (!e || !d || !c || !sd || !r || !slot) return ITOKMC_EINVAL;
  *slot = -1;
  if (!valid_desc(d)) return ens_error(e, ITOKMC_EINVAL, "invalid grid descriptor");
  if (d->field_mode != ITOKMC_FIELD_UNIFORM || d->n_ppc != 0 || d->precision != e->d.precision)
    return ens_error(e, ITOKMC_EINVAL,
                     "ensemble realizations need a uniform field, n_ppc 0 and the ensemble's precision");
  std::string why;
  if (check_coeffs(c, &why)) return ens_error(e, ITOKMC_EINVAL, "%s", why.c_str());
  if (c->beta_ep > 0.0 || c->beta_np > 0.0)
    return ens_error(e, ITOKMC_EINVAL, "the ensemble does not take recombination");
  if (c->mu_ion > 0.0 || c->D_ion > 0.0)
    return ens_error(e, ITOKMC_EINVAL, "the ensemble does not take mobile ions");
  if (c->kgamma_ratio != 0.0) return ens_error(e, ITOKMC_EINVAL, "ensemble realizations carry no photons");
  if (sd->kind != ITOKMC_SEED_GAUSSIAN || !(sd->sigma > 0.0))
    return ens_error(e, ITOKMC_EINVAL, "ensemble seeds are Gaussian electrons with sigma > 0");
  if (!(r->dt > 0.0) || r->nsteps < 1) return ens_error(e, ITOKMC_EINVAL, "dt > 0 and nsteps >= 1 required");
  if (sd->n0 > d->max_particles) return ens_error(e, ITOKMC_EINVAL, "seed exceeds the particle quota");
  const uint64_t ncell = (uint64_t)d->nx * d->ny * d->nz;
  const uint32_t nb = (uint32_t)((ncell + kBlkCells - 1) / kBlkCells);
  const uint64_t quota = d->max_particles;
  if (quota > e->cap || nb > e->nblk) return ens_error(e, ITOKMC_EINVAL, "realization larger than the pools");
  int s = -1;
  for (uint32_t i = 0; i < e->ms; ++i)
    if (!e->slots[i].used) { s = (int)i; break; }
  if (s < 0 || quota > e->quota_free || nb > e->free_blocks.size()) return ITOKMC_EAGAIN;
  uint32_t map_off = 0;
  if (!e->map_alloc.take(nb, &map_off)) return ITOKMC_EAGAIN;
  SlotHost& H = e->slots[s];
  H = SlotHost();
  H.used = true;
  H.d = *d;
  H.c = *c;
  H.r = *r;
  H.quota = quota;
  H.map_off = map_off;
  for (uint32_t i = 0; i < nb; ++i) {
    const uint32_t b = *e->free_blocks.begin();
    e->free_blocks.erase(e->free_blocks.begin());
    e->used_blocks.insert(b);
    H.blocks.push_back(b);
  }
  e->quota_free -= quota;
  SlotConst v{};
  v.nx = d->nx; v.ny = d->ny; v.nz = d->nz;
  v.ncell = (uint32_t)ncell;
  v.key = Key{d->seed, d->realization};
  v.step = 0;
  v.nsteps = r->nsteps;
  v.state = ITOKMC_SLOT_ACTIVE;
  v.n_new = (uint32_t)d->n_new;
  v.quota = (uint32_t)quota;
  v.map_off = map_off;
  v.stop = r->stop_particles;
  v.kp = KmcParams{d->kmc_mode, d->kmc_nc, d->kmc_nssa, d->kmc_eps};
  v.dt = r->dt;
  double k5[5];
  uniform_consts(*d, *c, r->dt, v.drift, &v.diff, k5);
  for (int i = 0; i < 3; ++i) v.k[i] = k5[i];
  hipError_t h = update_hw(e);
  if (h == hipSuccess) {
    e_set_slot<<<1, 64, 0, e->s>>>(v, s, e->sc, e->st, e->stat2, e->ms);
    h = hipGetLastError();
  }
  if (h == hipSuccess)
    h = for_lists(H.blocks, [&](const BlkList& L) {
      e_set_blocks<<<1, 256, 0, e->s>>>(L, s, map_off, e->blk_slot, e->blk_local, e->map);
      e_zero_cells<<<L.n, 256, 0, e->s>>>(L, e->nplus, e->nminus);
      return hipGetLastError();
    });
  if (h == hipSuccess && sd->n0 > 0) {
    const int g = (int)std::min<uint64_t>(4096, (sd->n0 + 255) / 256);
    if (f64(e))
      e_seed_gaussian<double><<<g, 256, 0, e->s>>>(e->bank[e->cur], e->ctr, e->cur, e->sc, s, e->map,
                                                   e->cap, sd->n0, d->dx, sd->centre[0], sd->centre[1],
                                                   sd->centre[2], sd->sigma);
    else
      e_seed_gaussian<float><<<g, 256, 0, e->s>>>(e->bank[e->cur], e->ctr, e->cur, e->sc, s, e->map,
                                                  e->cap, sd->n0, d->dx, sd->centre[0], sd->centre[1],
                                                  sd->centre[2], sd->sigma);
    h = hipGetLastError();
  }
  if (h != hipSuccess) return ens_hip(e, h, "admit");
  *slot = s;
  return ITOKMC_OK;
}

int itokmc_ensemble_step(itokmc_ens* e, uint32_t nsteps) {
  if (!e) return ITOKMC_EINVAL;
  const bool graph = e->tune.use_graph && capture_graphs(e);
  for (uint32_t i = 0; i < nsteps; ++i) {
    hipError_t h = graph ? hipGraphLaunch(e->graph[e->cur], e->s) : enqueue_step(e, e->cur, e->s);
    if (h != hipSuccess) return ens_hip(e, h, "ensemble step");
    e->cur = 1 - e->cur;
    e->steps += 1;
  }
  if (nsteps > 0 && (!e->pending_blocks.empty() || e->pending_quota || !e->pending_map.empty())) {
    // the step just enqueued dropped the particles of released slots
    for (uint32_t b : e->pending_blocks) e->free_blocks.insert(b);
    e->pending_blocks.clear();
    for (auto& m : e->pending_map) e->map_alloc.give(m.first, m.second);
    e->pending_map.clear();
    e->quota_free += e->pending_quota;
    e->pending_quota = 0;
    const hipError_t h = update_hw(e);
    if (h != hipSuccess) return ens_hip(e, h, "ensemble step");
  }
  return ITOKMC_OK;
}

int itokmc_ensemble_poll(itokmc_ens* e, itokmc_slot_event* ev, int32_t max, int32_t* n_ev) {
  if (!e || !n_ev || (max > 0 && !ev)) return ITOKMC_EINVAL;
  *n_ev = 0;
  uint32_t top = 0;
  for (uint32_t i = 0; i < e->ms; ++i)
    if (e->slots[i].used) top = i + 1;
  hipError_t h = hipSuccess;
  if (top) h = hipMemcpyAsync(e->host_stat, e->stat2, (size_t)top * 8, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipMemcpyAsync(e->host_ctr, e->ctr, sizeof(Counters), hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  if (h != hipSuccess) return ens_hip(e, h, "poll");
  int32_t k = 0;
  for (uint32_t i = 0; i < top && k < max; ++i) {
    SlotHost& H = e->slots[i];
    const uint32_t state = e->host_stat[2 * i];
    if (!H.used || H.reported || (state != ITOKMC_SLOT_DONE && state != ITOKMC_SLOT_CAPPED)) continue;
    H.reported = true;
    ev[k].slot = (int32_t)i;
    ev[k].state = (int32_t)state;
    ev[k].tag = H.r.tag;
    ev[k].steps = e->host_stat[2 * i + 1];
    ev[k].pad0 = 0;
    ++k;
  }
  *n_ev = k;
  if (e->host_ctr->overflow & ITOKMC_OVF_BARRIER)
    return ens_error(e, ITOKMC_EHIP,
                     "fused ensemble step: a device-wide barrier timed out; the ensemble's state is not valid");
  if (e->host_ctr->overflow)
    return ens_error(e, ITOKMC_ECAPACITY, "ensemble pool overflow (flags %u)", e->host_ctr->overflow);
  return ITOKMC_OK;
}

int itokmc_ensemble_results(itokmc_ens* e, const int32_t* slots, int32_t n, itokmc_diag* out) {
  if (!e || n < 0 || (n > 0 && (!slots || !out))) return ITOKMC_EINVAL;
  for (int32_t i = 0; i < n; ++i) {
    const int rc = check_slot(e, slots[i]);
    if (rc) return rc;
  }
  if (n == 0) return ITOKMC_OK;
  const size_t ms = e->ms;
  unsigned long long* pool = e->slot_red;           // 2 per slot (all slots)
  unsigned long long* ions = e->slot_red + 2 * ms;  // 2 per requested index
  hipError_t h = hipMemsetAsync(e->slot_red, 0, ms * 4 * 8, e->s);
  if (h == hipSuccess) {
    const int g = (int)std::min<uint64_t>(4096, ((uint64_t)e->cap + 255) / 256);
    e_reduce_all<<<g, 256, 0, e->s>>>(e->bank[e->cur], e->ctr, e->cur, e->cap, e->blk_slot, pool);
    h = hipGetLastError();
  }
  // ion sums: every block of every requested slot, tagged with the request index
  std::vector<uint32_t> blocks, tags;
  for (int32_t i = 0; i < n && h == hipSuccess; ++i)
    for (uint32_t b : e->slots[slots[i]].blocks) { blocks.push_back(b); tags.push_back((uint32_t)i); }
  for (size_t i = 0; i < blocks.size() && h == hipSuccess; i += kListMax) {
    BlkList L, T;
    L.n = T.n = (uint32_t)std::min<size_t>(kListMax, blocks.size() - i);
    L.first_local = T.first_local = 0;
    for (uint32_t k = 0; k < L.n; ++k) { L.b[k] = blocks[i + k]; T.b[k] = tags[i + k]; }
    e_reduce_ions_multi<<<L.n, 256, 0, e->s>>>(L, T, e->nplus, e->nminus, ions);
    h = hipGetLastError();
  }
  std::vector<unsigned long long> stv((size_t)S_NUM * ms), red(4 * ms);
  std::vector<uint32_t> st2(2 * ms);
  if (h == hipSuccess) h = hipMemcpyAsync(stv.data(), e->st, stv.size() * 8, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipMemcpyAsync(st2.data(), e->stat2, st2.size() * 4, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipMemcpyAsync(red.data(), e->slot_red, red.size() * 8, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  if (h != hipSuccess) return ens_hip(e, h, "results");
  for (int32_t i = 0; i < n; ++i) {
    const size_t s = (size_t)slots[i];
    auto S = [&](int f) { return stv[(size_t)f * ms + s]; };
    itokmc_diag* o = out + i;
    memset(o, 0, sizeof(*o));
    o->n_particles = red[2 * s];
    o->weight = red[2 * s + 1];
    o->n_plus = (int64_t)red[2 * ms + 2 * i];
    o->n_minus = (int64_t)red[2 * ms + 2 * i + 1];
    o->charge = o->n_plus - (int64_t)o->weight - o->n_minus;
    o->outflow_weight = S(S_OUTW);
    o->fires[0] = S(S_F0);
    o->fires[1] = S(S_F1);
    o->fires[2] = S(S_F2);
    o->created = S(S_CREATED);
    o->removed_weight = S(S_REMOVED);
    o->step = st2[2 * s + 1];
    o->rho_sum = 1.602176634e-19 * (double)o->charge;
    o->overflow = S(S_CAPPED) ? 1u : 0u;
    o->particle_steps = S(S_PUSHED);
  }
  return ITOKMC_OK;
}

int itokmc_ensemble_result(itokmc_ens* e, int32_t slot, itokmc_diag* out) {
  return itokmc_ensemble_results(e, &slot, 1, out);
}

int itokmc_ensemble_get_particles(itokmc_ens* e, int32_t slot, uint64_t* n, uint32_t* cell,
                                  double* off, uint32_t* w, uint64_t* id) {
  int rc = check_slot(e, slot);
  if (rc) return rc;
  if (!n) return ITOKMC_EINVAL;
  const int o = 1 - e->cur;  // the other bank is free between steps
  hipError_t h = hipMemsetAsync(e->misc + 1, 0, 4, e->s);
  if (h == hipSuccess) {
    const int g = (int)std::min<uint64_t>(4096, ((uint64_t)e->cap + 255) / 256);
    if (f64(e))
      e_extract<double><<<g, 256, 0, e->s>>>(e->bank[e->cur], e->ctr, e->cur, e->cap, slot, e->blk_slot,
                                             e->blk_local, e->bank[o], e->misc + 1);
    else
      e_extract<float><<<g, 256, 0, e->s>>>(e->bank[e->cur], e->ctr, e->cur, e->cap, slot, e->blk_slot,
                                            e->blk_local, e->bank[o], e->misc + 1);
    h = hipGetLastError();
  }
  uint32_t cnt = 0;
  if (h == hipSuccess) h = hipMemcpyAsync(&cnt, e->misc + 1, 4, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  if (h != hipSuccess) return ens_hip(e, h, "get_particles");
  const bool want = cell || off || w || id;
  if (want && *n < cnt) {
    *n = cnt;
    return ens_error(e, ITOKMC_EINVAL, "output arrays hold fewer than %u particles", cnt);
  }
  *n = cnt;
  if (!want || cnt == 0) return ITOKMC_OK;
  const Bank& B = e->bank[o];
  if (cell) h = hipMemcpyAsync(cell, B.cell, (size_t)cnt * 4, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess && w) h = hipMemcpyAsync(w, B.w, (size_t)cnt * 4, hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess && id) h = hipMemcpyAsync(id, B.id, (size_t)cnt * 8, hipMemcpyDeviceToHost, e->s);
  std::vector<char> tmp;
  if (h == hipSuccess && off) {
    const size_t T = f64(e) ? 8 : 4;
    tmp.resize((size_t)cnt * T * 3);
    void* src[3] = {B.ox, B.oy, B.oz};
    for (int a = 0; a < 3 && h == hipSuccess; ++a)
      h = hipMemcpyAsync(tmp.data() + (size_t)a * cnt * T, src[a], (size_t)cnt * T, hipMemcpyDeviceToHost, e->s);
  }
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  if (h != hipSuccess) return ens_hip(e, h, "get_particles");
  if (off) {
    for (uint32_t i = 0; i < cnt; ++i)
      for (int a = 0; a < 3; ++a)
        off[3 * (size_t)i + a] = f64(e) ? ((const double*)tmp.data())[(size_t)a * cnt + i]
                                        : (double)((const float*)tmp.data())[(size_t)a * cnt + i];
  }
  return ITOKMC_OK;
}

int itokmc_ensemble_get_counts(itokmc_ens* e, int32_t slot, int which, uint32_t* host) {
  int rc = check_slot(e, slot);
  if (rc) return rc;
  if (!host) return ITOKMC_EINVAL;
  const SlotHost& H = e->slots[slot];
  const uint64_t ncell = (uint64_t)H.d.nx * H.d.ny * H.d.nz;
  if (which == ITOKMC_Q_NGP_WEIGHT) {
    uint64_t n = 0;
    rc = itokmc_ensemble_get_particles(e, slot, &n, nullptr, nullptr, nullptr, nullptr);
    if (rc) return rc;
    std::vector<uint32_t> cell(n), w(n);
    rc = itokmc_ensemble_get_particles(e, slot, &n, cell.data(), nullptr, w.data(), nullptr);
    if (rc) return rc;
    memset(host, 0, ncell * 4);
    for (uint64_t i = 0; i < n; ++i) host[cell[i]] += w[i];
    return ITOKMC_OK;
  }
  const uint32_t* src;
  if (which == ITOKMC_Q_NPLUS) src = e->nplus;
  else if (which == ITOKMC_Q_NMINUS) src = e->nminus;
  else return ens_error(e, ITOKMC_EINVAL, "unsupported count selector %d", which);
  hipError_t h = hipSuccess;
  for (size_t lb = 0; lb < H.blocks.size() && h == hipSuccess; ++lb) {
    const uint64_t c0 = (uint64_t)lb * kBlkCells;
    const uint64_t len = std::min<uint64_t>(kBlkCells, ncell - c0);
    h = hipMemcpyAsync(host + c0, src + ((size_t)H.blocks[lb] << kBlkShift), len * 4,
                       hipMemcpyDeviceToHost, e->s);
  }
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  return ens_hip(e, h, "get_counts");
}

int itokmc_ensemble_release(itokmc_ens* e, int32_t slot) {
  int rc = check_slot(e, slot);
  if (rc) return rc;
  SlotHost& H = e->slots[slot];
  const hipError_t h = for_lists(H.blocks, [&](const BlkList& L) {
    e_clear_blocks<<<1, 256, 0, e->s>>>(L, L.first_local == 0 ? slot : -1, e->sc, e->stat2, e->blk_slot);
    return hipGetLastError();
  });
  if (h != hipSuccess) return ens_hip(e, h, "release");
  for (uint32_t b : H.blocks) {
    e->used_blocks.erase(b);
    e->pending_blocks.push_back(b);
  }
  e->pending_map.push_back({H.map_off, (uint32_t)H.blocks.size()});
  e->pending_quota += H.quota;
  H = SlotHost();
  return ITOKMC_OK;
}

int itokmc_ensemble_info(itokmc_ens* e, itokmc_ens_info* out) {
  if (!e || !out) return ITOKMC_EINVAL;
  hipError_t h = hipMemcpyAsync(e->host_ctr, e->ctr, sizeof(Counters), hipMemcpyDeviceToHost, e->s);
  if (h == hipSuccess) h = hipStreamSynchronize(e->s);
  if (h != hipSuccess) return ens_hip(e, h, "info");
  memset(out, 0, sizeof(*out));
  for (uint32_t i = 0; i < e->ms; ++i) {
    if (e->slots[i].used) out->slots_used += 1;
  }
  out->slots_free = (int32_t)e->ms - out->slots_used;
  out->cells_free = (uint64_t)e->free_blocks.size() * kBlkCells;
  out->particles_free = e->quota_free;
  out->pool_particles = std::min<uint64_t>(e->host_ctr->n[e->cur], e->cap);
  out->steps = e->steps;
  return ITOKMC_OK;
}

int itokmc_ensemble_set_tuning(itokmc_ens* e, const itokmc_ens_tuning* t) {
  if (!e || !t) return ITOKMC_EINVAL;
  if (t->push_block < 64 || t->push_block > 1024 || t->push_block % 64 ||
      t->push_blocks_per_cu < 1 || t->push_blocks_per_cu > 64 ||
      (t->kmc_block != 64 && t->kmc_block != 128 && t->kmc_block != 256) ||
      t->couple_per_cu < 1 || t->couple_per_cu > 256 ||
      (t->fused_per_cu != 0 && t->fused_per_cu != 1 && t->fused_per_cu != 2 && t->fused_per_cu != 4))
    return ens_error(e, ITOKMC_EINVAL, "tuning out of range");
  if (t->fused_per_cu && !(e->fuse_occ & t->fused_per_cu))
    return ens_error(e, ITOKMC_EINVAL,
                     "fused step: %d workgroups per compute unit do not stay resident on this device",
                     t->fused_per_cu);
  e->tune = *t;
  drop_graphs(e);
  return ITOKMC_OK;
}

int itokmc_ensemble_get_tuning(itokmc_ens* e, itokmc_ens_tuning* t) {
  if (!e || !t) return ITOKMC_EINVAL;
  *t = e->tune;
  return ITOKMC_OK;
}

int itokmc_ensemble_autotune(itokmc_ens* e, uint32_t rounds, itokmc_ens_tuning* best,
                             double* best_ms) {
  if (!e || rounds < 1) return ITOKMC_EINVAL;
  const itokmc_ens_tuning base = e->tune;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return ens_error(e, ITOKMC_EHIP, "autotune: event creation failed");
  // coordinate search: particle-kernel shape, then KMC block, then coupling grid
  itokmc_ens_tuning cur = base;
  double cur_ms = 0.0;
  int rc = ITOKMC_OK;
  auto measure = [&](const std::vector<itokmc_ens_tuning>& cands, size_t* arg, double* ms) -> int {
    std::vector<double> tot(cands.size(), 0.0);
    for (uint32_t r = 0; r < rounds; ++r) {
      for (size_t i = 0; i < cands.size(); ++i) {
        int q = itokmc_ensemble_set_tuning(e, &cands[i]);
        if (q) return q;
        if (e->tune.use_graph && !capture_graphs(e)) return ens_error(e, ITOKMC_EHIP, "autotune: capture failed");
        if (hipEventRecord(e0, e->s) != hipSuccess) return ens_error(e, ITOKMC_EHIP, "autotune: event");
        q = itokmc_ensemble_step(e, 1);
        if (q) return q;
        if (hipEventRecord(e1, e->s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
          return ens_error(e, ITOKMC_EHIP, "autotune: event");
        float m = 0.f;
        (void)hipEventElapsedTime(&m, e0, e1);
        tot[i] += m;
      }
    }
    *arg = (size_t)(std::min_element(tot.begin(), tot.end()) - tot.begin());
    *ms = tot[*arg] / rounds;
    return ITOKMC_OK;
  };
  std::vector<itokmc_ens_tuning> c1;
  for (int pb : {256, 512, 1024})
    for (int pc : {2, 4, 8, 16}) {
      itokmc_ens_tuning t = cur;
      t.push_block = pb;
      t.push_blocks_per_cu = pc;
      c1.push_back(t);
    }
  size_t arg = 0;
  rc = measure(c1, &arg, &cur_ms);
  if (!rc) {
    cur = c1[arg];
    std::vector<itokmc_ens_tuning> c2;
    for (int kb : {64, 128, 256}) { itokmc_ens_tuning t = cur; t.kmc_block = kb; c2.push_back(t); }
    rc = measure(c2, &arg, &cur_ms);
    if (!rc) cur = c2[arg];
  }
  if (!rc) {
    std::vector<itokmc_ens_tuning> c3;
    for (int cc : {16, 64, 256}) { itokmc_ens_tuning t = cur; t.couple_per_cu = cc; c3.push_back(t); }
    rc = measure(c3, &arg, &cur_ms);
    if (!rc) cur = c3[arg];
  }
  if (!rc) {
    // the form of the step: the kernel sequence (with the shapes found above) against
    // the persistent fused kernel at each resident grid size
    std::vector<itokmc_ens_tuning> c4;
    for (int k : {0, 1, 2, 4}) {
      if (k && !(e->fuse_occ & k)) continue;
      itokmc_ens_tuning t = cur;
      t.fused_per_cu = k;
      c4.push_back(t);
    }
    rc = measure(c4, &arg, &cur_ms);
    if (!rc) cur = c4[arg];
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc) {
    (void)itokmc_ensemble_set_tuning(e, &base);
    return rc;
  }
  rc = itokmc_ensemble_set_tuning(e, &cur);
  if (best) *best = cur;
  if (best_ms) *best_ms = cur_ms;
  return rc;
}

void itokmc_ensemble_destroy(itokmc_ens* e) {
  if (!e) return;
  (void)hipStreamSynchronize(e->s);
  drop_graphs(e);
  if (e->host_stat) (void)hipHostFree(e->host_stat);
  if (e->host_ctr) (void)hipHostFree(e->host_ctr);
  if (e->host_red) (void)hipHostFree(e->host_red);
  delete e;
}

const char* itokmc_ensemble_last_error(const itokmc_ens* e) {
  return e ? e->err.c_str() : "null ensemble";
}

}  // extern "C"
