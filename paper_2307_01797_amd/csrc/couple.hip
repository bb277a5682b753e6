// KMC-particle coupling (section "KMC-particle coupling", eq. w): one wavefront per
// queued cell.  A net gain dN > 0 becomes min(dN, n_new) new particles of weight
// dN div M, the remainder going to the first, placed uniformly in the cell and
// appended to the bank; a net loss removes weight from the cell's particles in
// ascending id order (a particle reaching weight 0 is dead and dropped by the next
// binning).  Superparticle management (merge/split to n_ppc per cell) is applied to
// the cell afterwards when enabled.
#include <math.h>

#include "device.hpp"
#include "itk.hpp"
#include "couple_device.hpp"
#include "merge.hpp"

namespace itk {

namespace {

template <typename T>
__device__ __forceinline__ T* as(void* p) { return reinterpret_cast<T*>(p); }

template <typename T>
__global__ void __launch_bounds__(64) k_couple(Bank b, Counters* ctr, int which, StepConst K,
                                              const uint32_t* work, const uint32_t* occ,
                                              const uint32_t* start, const int32_t* dN,
                                              const uint32_t* cbase, int n_new, int n_ppc,
                                              uint32_t* big) {
  const uint32_t nwork = ctr->n_work, n_occ = ctr->n_occ, sorted = ctr->sorted;
  const int lane = lane_id();
  uint64_t created = 0, removed = 0, merged = 0;
  for (uint32_t t = blockIdx.x; t < nwork; t += gridDim.x) {
    const uint32_t j = work[t];
    const uint32_t c = occ[j];
    // the cell's sorted range ends where the next occupied cell's begins
    const uint32_t s = start[c], e = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
    const int32_t d = dN[j];
    if (d < 0) removed += remove_weight(b, s, e, (uint32_t)(-d));
    uint32_t M = 0, wb = 0, wr = 0, base = 0;
    if (d > 0) {
      M = (uint32_t)d < (uint32_t)n_new ? (uint32_t)d : (uint32_t)n_new;
      wb = (uint32_t)d / M;
      wr = (uint32_t)d % M;
      base = cbase[j];  // slots reserved by the KMC pass
    }
    // new particles, one per lane (n_new <= 64), into the reserved slots
    if ((uint32_t)lane < M) {
      const uint32_t q = base + (uint32_t)lane;
      if (q < K.cap) write_product<T>(b, q, c, c, (uint32_t)lane, wb, wr, K.step, K.key);
      else atomicOr(&ctr->overflow, 1u);
    }
    created += M;
    if (n_ppc > 0) {
      __syncthreads();  // removal and product stores visible before the merge gathers them
      const int r = merge_cell<T, kMergeTiny>(b, ctr, which, K, c, s, e, base, M, n_ppc, &merged);
      if (r == 2 && lane == 0) big[atomicAdd(&ctr->n_big, 1u)] = j;
    }
  }
  if (lane == 0) {
    if (created) atomicAdd(&ctr->created, (unsigned long long)created);
    if (removed) atomicAdd(&ctr->removed, (unsigned long long)removed);
    if (merged) atomicAdd(&ctr->merged, (unsigned long long)merged);
  }
}

// Cells whose particles exceed a staging area, merged with the next larger one:
// tier CAP reads its cells from list `in` (count *n_in); cells exceeding CAP go to
// list `out` (count *n_out) or, from the largest tier, are left unmerged and counted.
template <typename T, int CAP>
__global__ void __launch_bounds__(64) k_merge_tier(Bank b, Counters* ctr, int which, StepConst K,
                                                  const uint32_t* in, const uint32_t* n_in,
                                                  uint32_t* out, uint32_t* n_out,
                                                  const uint32_t* occ, const uint32_t* start,
                                                  const int32_t* dN, const uint32_t* cbase,
                                                  int n_new, int n_ppc) {
  const uint32_t nin = *n_in, n_occ = ctr->n_occ, sorted = ctr->sorted;
  uint64_t merged = 0;
  for (uint32_t t = blockIdx.x; t < nin; t += gridDim.x) {
    const uint32_t j = in[t];
    const uint32_t c = occ[j];
    const int32_t d = dN[j];
    const uint32_t M = d > 0 ? ((uint32_t)d < (uint32_t)n_new ? (uint32_t)d : (uint32_t)n_new) : 0u;
    const uint32_t base = M ? cbase[j] : 0u;
    const uint32_t e = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
    const int r = merge_cell<T, CAP>(b, ctr, which, K, c, start[c], e, base, M, n_ppc, &merged);
    if (r == 2 && lane_id() == 0) {
      if (out) out[atomicAdd(n_out, 1u)] = j;
      else atomicAdd(&ctr->merge_skipped, 1u);
    }
  }
  if (lane_id() == 0 && merged) atomicAdd(&ctr->merged, (unsigned long long)merged);
}

}  // namespace

hipError_t launch_couple(itokmc_ctx* ctx, const StepConst& k) {
  const int dest = 1 - ctx->cur;  // coupling acts on the freshly binned bank
  int g = (int)(ctx->ncell < 65536u ? ctx->ncell : 65536u);
  if (g < 1) g = 1;
  const bool f64 = ctx->d.precision == ITOKMC_FP64;
  if (f64)
    k_couple<double><<<g, 64, merge_lds_bytes<double>(ctx->d.n_ppc), ctx->s>>>(
        ctx->bank[dest], ctx->ctr, dest, k, ctx->work, ctx->occ, ctx->start, ctx->dN, ctx->cbase,
        ctx->d.n_new, ctx->d.n_ppc, ctx->big);
  else
    k_couple<float><<<g, 64, merge_lds_bytes<float>(ctx->d.n_ppc), ctx->s>>>(
        ctx->bank[dest], ctx->ctr, dest, k, ctx->work, ctx->occ, ctx->start, ctx->dN, ctx->cbase,
        ctx->d.n_new, ctx->d.n_ppc, ctx->big);
  hipError_t e = hipGetLastError();
  phase_end(ctx, PH_COUPLE);
  if (e != hipSuccess || ctx->d.n_ppc == 0) return e;
  phase_begin(ctx, PH_MERGE);  // the larger merge tiers
  Counters* C = ctx->ctr;
  if (f64) {
    k_merge_tier<double, kMergeSmall><<<2048, 64, merge_lds_bytes_c<double, kMergeSmall>(), ctx->s>>>(
        ctx->bank[dest], C, dest, k, ctx->big, &C->n_big, ctx->huge, &C->n_huge, ctx->occ, ctx->start,
        ctx->dN, ctx->cbase, ctx->d.n_new, ctx->d.n_ppc);
    k_merge_tier<double, MergeBig<double>::value>
        <<<1024, 64, merge_lds_bytes_c<double, MergeBig<double>::value>(), ctx->s>>>(
            ctx->bank[dest], C, dest, k, ctx->huge, &C->n_huge, nullptr, nullptr, ctx->occ, ctx->start,
            ctx->dN, ctx->cbase, ctx->d.n_new, ctx->d.n_ppc);
  } else {
    k_merge_tier<float, kMergeSmall><<<2048, 64, merge_lds_bytes_c<float, kMergeSmall>(), ctx->s>>>(
        ctx->bank[dest], C, dest, k, ctx->big, &C->n_big, ctx->huge, &C->n_huge, ctx->occ, ctx->start,
        ctx->dN, ctx->cbase, ctx->d.n_new, ctx->d.n_ppc);
    k_merge_tier<float, MergeBig<float>::value>
        <<<1024, 64, merge_lds_bytes_c<float, MergeBig<float>::value>(), ctx->s>>>(
            ctx->bank[dest], C, dest, k, ctx->huge, &C->n_huge, nullptr, nullptr, ctx->occ, ctx->start,
            ctx->dN, ctx->cbase, ctx->d.n_new, ctx->d.n_ppc);
  }
  phase_end(ctx, PH_MERGE);
  return hipGetLastError();
}

}  // namespace itk
