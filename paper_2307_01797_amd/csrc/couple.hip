// KMC-particle coupling (section "KMC-particle coupling", eq. w).  A net gain dN > 0
// becomes min(dN, n_new) new particles of weight dN div M, the remainder going to the
// first, placed uniformly in the cell and appended to the bank; a net loss removes
// weight from the cell's particles in ascending id order (a particle reaching weight 0
// is dead and dropped by the next binning).  Superparticle management (merge/split to
// n_ppc per cell) is applied to the cell afterwards when enabled.
//
// Most queued cells hold a handful of particles.  A light pass takes one cell per lane:
// it does the removal and the products of cells with at most kLightMax particles and
// products, checks whether they need merging or splitting, and queues the cells that
// do (merge only) and the larger cells (everything) for the wavefront-per-cell pass.
// The arithmetic and its order are the same on both paths.
#include <math.h>

#include <type_traits>

#include "device.hpp"
#include "itk.hpp"
#include "couple_device.hpp"
#include "merge.hpp"

namespace itk {

namespace {

template <typename T>
__device__ __forceinline__ T* as(void* p) { return reinterpret_cast<T*>(p); }

constexpr uint32_t kLightMax = 16;

template <typename T>
__global__ void __launch_bounds__(256) k_couple_light(Bank b, Counters* ctr, StepConst K,
                                                     const uint32_t* work, const uint32_t* occ,
                                                     const uint32_t* start, const int32_t* dN,
                                                     const uint32_t* cbase, int n_new, int n_ppc,
                                                     uint32_t* full_list, uint32_t* merge_list) {
  if (ctr->halt) return;
  __shared__ uint32_t sh[18];
  const uint32_t nwork = ctr->n_work, n_occ = ctr->n_occ, sorted = ctr->sorted;
  uint64_t created = 0, removed = 0;
  for (uint32_t base = blockIdx.x * blockDim.x; base < nwork; base += gridDim.x * blockDim.x) {
    const uint32_t t = base + threadIdx.x;
    bool to_full = false, to_merge = false;
    uint32_t j = 0;
    if (t < nwork) {
      j = work[t];
      const uint32_t c = occ[j];
      const uint32_t s = start[c], e = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
      const int32_t d = dN[j];
      const uint32_t M = d > 0 ? ((uint32_t)d < (uint32_t)n_new ? (uint32_t)d : (uint32_t)n_new) : 0u;
      if (e - s > kLightMax || M > kLightMax) {
        to_full = true;
      } else {
        if (d < 0) removed += remove_weight_lane(b, s, e, (uint32_t)(-d));
        uint32_t wb = 0, wr = 0, pb = 0;
        if (M) {
          wb = (uint32_t)d / M;
          wr = (uint32_t)d % M;
          pb = cbase[j];
          for (uint32_t k = 0; k < M; ++k) {
            const uint32_t q = pb + k;
            if (q < K.cap) write_product<T>(b, q, c, c, k, wb, wr, K.step, K.key);
            else atomicOr(&ctr->overflow, 1u);
          }
          created += M;
        }
        if (n_ppc > 0) {  // the merge trigger, as merge_cell evaluates it
          uint32_t m = 0, wmax = 0;
          for (uint32_t q = s; q < e; ++q) {
            const uint32_t w = b.w[q];
            if (w > 0) { ++m; wmax = w > wmax ? w : wmax; }
          }
          if (M) {
            m += M;
            const uint32_t w0 = wb + wr;
            wmax = w0 > wmax ? w0 : wmax;
          }
          to_merge = m > 0 && (m > (uint32_t)n_ppc || (m < (uint32_t)n_ppc && wmax >= 2));
        }
      }
    }
    const uint32_t qf = block_append(&ctr->n_cfull, to_full ? 1u : 0u, sh);
    if (to_full) full_list[qf] = j;
    const uint32_t qm = block_append(&ctr->n_cmerge, to_merge ? 1u : 0u, sh);
    if (to_merge) merge_list[qm] = j;
  }
  created = wave_sum64(created);
  removed = wave_sum64(removed);
  if (lane_id() == 0) {
    if (created) atomicAdd(&ctr->created, (unsigned long long)created);
    if (removed) atomicAdd(&ctr->removed, (unsigned long long)removed);
  }
}

// One wavefront per cell: the cells of full_list (removal, products, merge) and then
// those of merge_list (merge only; the light pass did the rest).
template <typename T, int NL>
__global__ void __launch_bounds__(64, 5) k_couple(Bank b, Counters* ctr, int which, StepConst K,
                                              const uint32_t* full_list, const uint32_t* merge_list,
                                              const uint32_t* occ, const uint32_t* start,
                                              const int32_t* dN, const uint32_t* cbase, int n_new,
                                              int n_ppc, uint32_t* big) {
  if (ctr->halt) return;
  const uint32_t nfull = ctr->n_cfull, nwork = nfull + ctr->n_cmerge, n_occ = ctr->n_occ,
                 sorted = ctr->sorted;
  const int lane = lane_id();
  uint64_t created = 0, removed = 0, merged = 0, pieces = 0;
  for (uint32_t t = blockIdx.x; t < nwork; t += gridDim.x) {
    const bool full = t < nfull;
    const uint32_t j = full ? full_list[t] : merge_list[t - nfull];
    const uint32_t c = occ[j];
    // the cell's sorted range ends where the next occupied cell's begins
    const uint32_t s = start[c], e = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
    const int32_t d = dN[j];
    if (full && d < 0) removed += remove_weight(b, s, e, (uint32_t)(-d));
    uint32_t M = 0, wb = 0, wr = 0, base = 0;
    if (d > 0) {
      M = (uint32_t)d < (uint32_t)n_new ? (uint32_t)d : (uint32_t)n_new;
      wb = (uint32_t)d / M;
      wr = (uint32_t)d % M;
      base = cbase[j];  // slots reserved by the KMC pass
    }
    // new particles, one per lane (n_new <= 64), for the reserved slots; slots past the
    // bank's capacity are flagged
    const bool mine = full && (uint32_t)lane < M;
    const uint32_t q = base + (uint32_t)lane;
    if (mine && q >= K.cap) atomicOr(&ctr->overflow, 1u);
    if (full) created += M;
    pieces += (e - s) + M;
    int r = 0;
    if (n_ppc > 0) {
      // removal stores visible before the merge gathers the cell (nothing to wait for
      // otherwise: the previous cell's leaf stores are to other slots); the products
      // are made by the gather itself and stored only if the cell is not merged here
      if (full && d < 0) __syncthreads();
      else wave_lds_sync();
      r = merge_cell<T, kMergeTiny, NL>(b, ctr, which, K, c, s, e, base, M, n_ppc, &merged, full, wb, wr);
      if (r == 2 && lane == 0) big[atomicAdd(&ctr->n_big, 1u)] = j;
    }
    if (mine && r != 1 && q < K.cap) write_product<T>(b, q, c, c, (uint32_t)lane, wb, wr, K.step, K.key);
  }
  if (lane == 0) {
    if (created) atomicAdd(&ctr->created, (unsigned long long)created);
    if (removed) atomicAdd(&ctr->removed, (unsigned long long)removed);
    if (merged) atomicAdd(&ctr->merged, (unsigned long long)merged);
    if (pieces) atomicAdd(&ctr->couple_pieces, (unsigned long long)pieces);
  }
}

// Cells whose particles exceed a staging area, merged with the next larger one:
// tier CAP reads its cells from list `in` (count *n_in); cells exceeding CAP go to
// list `out` (count *n_out) or, from the largest tier, are left unmerged and counted.
template <typename T, int CAP, int NL>
__global__ void __launch_bounds__(64) k_merge_tier(Bank b, Counters* ctr, int which, StepConst K,
                                                  const uint32_t* in, const uint32_t* n_in,
                                                  uint32_t* out, uint32_t* n_out,
                                                  const uint32_t* occ, const uint32_t* start,
                                                  const int32_t* dN, const uint32_t* cbase,
                                                  int n_new, int n_ppc) {
  if (ctr->halt) return;
  const uint32_t nin = *n_in, n_occ = ctr->n_occ, sorted = ctr->sorted;
  uint64_t merged = 0;
  for (uint32_t t = blockIdx.x; t < nin; t += gridDim.x) {
    const uint32_t j = in[t];
    const uint32_t c = occ[j];
    const int32_t d = dN[j];
    const uint32_t M = d > 0 ? ((uint32_t)d < (uint32_t)n_new ? (uint32_t)d : (uint32_t)n_new) : 0u;
    const uint32_t base = M ? cbase[j] : 0u;
    const uint32_t e = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
    const int r = merge_cell<T, CAP, NL>(b, ctr, which, K, c, start[c], e, base, M, n_ppc, &merged);
    if (r == 2 && lane_id() == 0) {
      if (out) out[atomicAdd(n_out, 1u)] = j;
      else {  // larger than every staging: left unmerged, reported as ECAPACITY
        atomicAdd(&ctr->merge_skipped, 1u);
        atomicOr(&ctr->overflow, (uint32_t)ITOKMC_OVF_MERGE);
      }
    }
  }
  if (lane_id() == 0 && merged) atomicAdd(&ctr->merged, (unsigned long long)merged);
}

}  // namespace

hipError_t launch_couple(itokmc_ctx* ctx, const StepConst& k) {
  const int dest = 1 - ctx->cur;  // coupling acts on the freshly binned bank
  const bool f64 = ctx->d.precision == ITOKMC_FP64;
  int gl = (int)((ctx->ncell + 255) / 256);
  // at most 768 workgroups (three per CU), each looping over the queue: 0.096 ms per
  // step at 9.5e6 particles against 0.21 ms with 4096 and 0.125 ms with 256
  gl = gl < 1 ? 1 : (gl > 768 ? 768 : gl);
  if (f64)
    k_couple_light<double><<<gl, 256, 0, ctx->s>>>(ctx->bank[dest], ctx->ctr, k, ctx->work, ctx->occ,
                                                   ctx->start, ctx->dN, ctx->cbase, ctx->d.n_new,
                                                   ctx->d.n_ppc, ctx->cfull, ctx->cmerge);
  else
    k_couple_light<float><<<gl, 256, 0, ctx->s>>>(ctx->bank[dest], ctx->ctr, k, ctx->work, ctx->occ,
                                                  ctx->start, ctx->dN, ctx->cbase, ctx->d.n_new,
                                                  ctx->d.n_ppc, ctx->cfull, ctx->cmerge);
  hipError_t el = hipGetLastError();
  phase_end(ctx, PH_COUPLE_LIGHT);
  if (el != hipSuccess) return el;
  phase_begin(ctx, PH_COUPLE);  // the wavefront-per-cell kernel alone
  // a grid of 32768 one-wavefront workgroups (128 per CU), each taking every 32768th
  // queued cell: measured at 1.82 ms per launch at 9.5e6 particles, against 2.17 ms with
  // 65536, 3.5 ms with 131072 and 2.05 ms with 10240 workgroups (28672-49152 all within
  // 1%)
  int g = (int)(ctx->ncell < 32768u ? ctx->ncell : 32768u);
  if (g < 1) g = 1;
  const int nl = merge_leaves(ctx->d.n_ppc);
  auto wave = [&](auto tt, auto nlt) {
    using T = decltype(tt);
    constexpr int NL = decltype(nlt)::value;
    const size_t lds = ctx->d.n_ppc > 0 ? merge_lds_bytes_c<T, kMergeTiny, NL>() : 0;
    k_couple<T, NL><<<g, 64, lds, ctx->s>>>(ctx->bank[dest], ctx->ctr, dest, k, ctx->cfull, ctx->cmerge,
                                          ctx->occ, ctx->start, ctx->dN, ctx->cbase, ctx->d.n_new,
                                          ctx->d.n_ppc, ctx->big);
  };
  using N32 = std::integral_constant<int, 32>;
  using N64 = std::integral_constant<int, kMaxMergePpc>;
  if (f64) { if (nl == 32) wave(0.0, N32{}); else wave(0.0, N64{}); }
  else { if (nl == 32) wave(0.0f, N32{}); else wave(0.0f, N64{}); }
  hipError_t e = hipGetLastError();
  phase_end(ctx, PH_COUPLE);
  if (e != hipSuccess || ctx->d.n_ppc == 0) return e;
  phase_begin(ctx, PH_MERGE);  // the larger merge tiers
  Counters* C = ctx->ctr;
  auto tiers = [&](auto tt, auto nlt) {
    using T = decltype(tt);
    constexpr int NL = decltype(nlt)::value;
    constexpr int BIG = MergeBig<T>::value;
    k_merge_tier<T, kMergeSmall, NL><<<2048, 64, merge_lds_bytes_c<T, kMergeSmall, NL>(), ctx->s>>>(
        ctx->bank[dest], C, dest, k, ctx->big, &C->n_big, ctx->huge, &C->n_huge, ctx->occ, ctx->start,
        ctx->dN, ctx->cbase, ctx->d.n_new, ctx->d.n_ppc);
    k_merge_tier<T, BIG, NL><<<1024, 64, merge_lds_bytes_c<T, BIG, NL>(), ctx->s>>>(
        ctx->bank[dest], C, dest, k, ctx->huge, &C->n_huge, nullptr, nullptr, ctx->occ, ctx->start,
        ctx->dN, ctx->cbase, ctx->d.n_new, ctx->d.n_ppc);
  };
  if (f64) { if (nl == 32) tiers(0.0, N32{}); else tiers(0.0, N64{}); }
  else { if (nl == 32) tiers(0.0f, N32{}); else tiers(0.0f, N64{}); }
  phase_end(ctx, PH_MERGE);
  return hipGetLastError();
}

}  // namespace itk
