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
      const int r = merge_cell<T, kMergeSmall>(b, ctr, which, K, c, s, e, base, M, n_ppc, &merged);
      if (r == 2 && lane == 0) big[atomicAdd(&ctr->n_big, 1u)] = j;
    }
  }
  if (lane == 0) {
    if (created) atomicAdd(&ctr->created, (unsigned long long)created);
    if (removed) atomicAdd(&ctr->removed, (unsigned long long)removed);
    if (merged) atomicAdd(&ctr->merged, (unsigned long long)merged);
  }
}

// Cells whose particles exceed the small staging area, merged with the large one.
template <typename T>
__global__ void __launch_bounds__(64) k_merge_big(Bank b, Counters* ctr, int which, StepConst K,
                                                 const uint32_t* big, const uint32_t* occ,
                                                 const uint32_t* start, const int32_t* dN,
                                                 const uint32_t* cbase, int n_new, int n_ppc) {
  const uint32_t nbig = ctr->n_big, n_occ = ctr->n_occ, sorted = ctr->sorted;
  uint64_t merged = 0;
  for (uint32_t t = blockIdx.x; t < nbig; t += gridDim.x) {
    const uint32_t j = big[t];
    const uint32_t c = occ[j];
    const int32_t d = dN[j];
    const uint32_t M = d > 0 ? ((uint32_t)d < (uint32_t)n_new ? (uint32_t)d : (uint32_t)n_new) : 0u;
    const uint32_t base = M ? cbase[j] : 0u;
    const uint32_t e = j + 1 < n_occ ? start[occ[j + 1]] : sorted;
    const int r = merge_cell<T, MergeBig<T>::value>(b, ctr, which, K, c, start[c], e, base, M, n_ppc,
                                                     &merged);
    if (r == 2 && lane_id() == 0) atomicAdd(&ctr->merge_skipped, 1u);
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
  if (e != hipSuccess || ctx->d.n_ppc == 0) return e;
  const int gb = 1024;
  if (f64) {
    const size_t lds = merge_lds_bytes_c<double, MergeBig<double>::value>();
    k_merge_big<double><<<gb, 64, lds, ctx->s>>>(ctx->bank[dest], ctx->ctr, dest, k, ctx->big, ctx->occ,
                                                  ctx->start, ctx->dN, ctx->cbase, ctx->d.n_new,
                                                  ctx->d.n_ppc);
  } else {
    const size_t lds = merge_lds_bytes_c<float, MergeBig<float>::value>();
    k_merge_big<float><<<gb, 64, lds, ctx->s>>>(ctx->bank[dest], ctx->ctr, dest, k, ctx->big, ctx->occ,
                                                 ctx->start, ctx->dN, ctx->cbase, ctx->d.n_new,
                                                 ctx->d.n_ppc);
  }
  return hipGetLastError();
}

}  // namespace itk
