// KMC-particle coupling device code shared by the single-realization and the ensemble
// kernels (see couple.hip).
#pragma once
#include "device.hpp"
#include "itk.hpp"

namespace itk {

// Remove R weight from particles [s, e) of bank b in ascending id order.
__device__ inline uint64_t remove_weight(Bank b, uint32_t s, uint32_t e, uint32_t R) {
  const int lane = lane_id();
  uint64_t removed = 0;
  while (R > 0) {
    uint64_t best = ~0ull;
    uint32_t bi = 0xFFFFFFFFu;
    for (uint32_t q = s + lane; q < e; q += 64) {
      if (b.w[q] > 0) {
        const uint64_t id = b.id[q];
        if (id < best) { best = id; bi = q; }
      }
    }
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) {
      const uint64_t ob = (uint64_t)__shfl_xor((unsigned long long)best, d, 64);
      const uint32_t oi = __shfl_xor(bi, d, 64);
      if (ob < best) { best = ob; bi = oi; }
    }
    if (bi == 0xFFFFFFFFu) break;  // nothing left (not reachable: KMC keeps X_e >= 0)
    uint32_t take = 0;
    if (lane == 0) {
      const uint32_t w = b.w[bi];
      take = w < R ? w : R;
      b.w[bi] = w - take;
    }
    take = __shfl(take, 0, 64);
    // make lane 0's store visible to the whole wavefront before the next search
    __syncthreads();
    if (take == 0) break;  // no progress possible (cannot happen with consistent weights)
    R -= take;
    removed += take;
  }
  return removed;
}

// The same removal by one lane (cells with few particles): the smallest id first.
__device__ inline uint64_t remove_weight_lane(Bank b, uint32_t s, uint32_t e, uint32_t R) {
  uint64_t removed = 0;
  while (R > 0) {
    uint64_t best = ~0ull;
    uint32_t bi = 0xFFFFFFFFu;
    for (uint32_t q = s; q < e; ++q) {
      if (b.w[q] > 0) {
        const uint64_t id = b.id[q];
        if (id < best) { best = id; bi = q; }
      }
    }
    if (bi == 0xFFFFFFFFu) break;
    const uint32_t w = b.w[bi];
    const uint32_t take = w < R ? w : R;
    b.w[bi] = w - take;
    R -= take;
    removed += take;
  }
  return removed;
}

// The k-th of M KMC products of a cell (local index lc for ids and streams): offsets
// uniform in the cell, weight wb (+ wr for the first), id.
template <typename T>
struct Product {
  T o[3];
  uint32_t w;
  uint64_t id;
};
template <typename T>
__device__ __forceinline__ Product<T> make_product(uint32_t lc, uint32_t k, uint32_t wb, uint32_t wr,
                                                   uint32_t step, Key key) {
  const uint4 r = philox_block(lc, k, step, TAG_CREATE, 0, key);
  Product<T> p;
  p.o[0] = (T)u24(r.x);
  p.o[1] = (T)u24(r.y);
  p.o[2] = (T)u24(r.z);
  p.w = wb + (k == 0 ? wr : 0u);
  p.id = make_id(KIND_KMC, step, lc, k);
  return p;
}

// Write that product into bank slot q of global cell gcell.
template <typename T>
__device__ __forceinline__ void write_product(Bank b, uint32_t q, uint32_t gcell, uint32_t lc,
                                              uint32_t k, uint32_t wb, uint32_t wr, uint32_t step,
                                              Key key) {
  const Product<T> p = make_product<T>(lc, k, wb, wr, step, key);
  b.cell[q] = gcell;
  reinterpret_cast<T*>(b.ox)[q] = p.o[0];
  reinterpret_cast<T*>(b.oy)[q] = p.o[1];
  reinterpret_cast<T*>(b.oz)[q] = p.o[2];
  b.w[q] = p.w;
  b.id[q] = p.id;
}

}  // namespace itk
