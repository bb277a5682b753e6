// Superparticle merge/split of one cell by one wavefront (section "Superparticle
// management").  Placeholder interface; the tree build is added with its kernel.
#pragma once
#include "device.hpp"
#include "itk.hpp"

namespace itk {

struct MergeScratch {
  int dummy;
};

inline MergeScratch merge_scratch(itokmc_ctx*) { return MergeScratch{0}; }
template <typename T>
inline size_t merge_lds_bytes(int) { return 0; }

template <typename T>
__device__ bool merge_cell(Bank, Counters*, int, const StepConst&, uint32_t, uint32_t, uint32_t,
                           uint32_t, uint32_t, const T*, uint32_t, uint64_t, int,
                           const MergeScratch&, uint64_t*) {
  return false;
}

}  // namespace itk
