// Counting sort of particles by cell, as a kernel-level entry point: the binning step
// that groups each cell's computational particles (the per-cell particle lists that the
// reactions and the superparticle pass of the paper's final algorithm work on).
//
//   count:   per live particle (w > 0), a run-aggregated atomic on its cell's counter
//            returns the particle's rank inside the cell;
//   scan:    exclusive prefix of the counters over all cells gives start[0 .. ncell];
//   scatter: particle i goes to start[cell] + rank (no atomics).
// Within a cell the order is that of the counting atomics (unspecified).
//
// Scratch (32-bit words): the per-cell counters [ncell], the ranks [n] and the scan's
// block partials.  itokmc_sort_by_cell takes it from a caller workspace;
// itokmc_sort_by_cell_noalloc from a file-scope device array (one per GPU, resolved once
// per device with hipGetSymbolAddress), for callers that cannot allocate.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <mutex>

#include "device.hpp"
#include "itk.hpp"

namespace itk {
namespace {

constexpr int kSortBlock = 256;
constexpr int kSortPer = 8;                          // cells per thread in the scan
constexpr uint32_t kSortTile = kSortBlock * kSortPer;  // cells per scan block
constexpr int kSortTopThreads = 1024;

// Words of scratch for n particles and ncell cells.
inline uint64_t sort_words(uint64_t n, uint64_t ncell) {
  const uint64_t nblk = (ncell + kSortTile - 1) / kSortTile;
  auto al = [](uint64_t w) { return (w + 63) & ~(uint64_t)63; };  // 256-byte alignment
  return al(ncell) + al(n) + al(nblk + 2);
}

__global__ void k_sort_fill(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

// Run-aggregated 32-bit atomic increment: lanes whose keys form a run (particles are
// usually grouped by cell already) take one atomic per run; each active lane gets the
// counter's value before its own increment.
__device__ __forceinline__ uint32_t run_inc(uint32_t* acc, uint32_t key) {
  const int lane = lane_id();
  const bool active = key != kInvalidCell;
  const uint32_t prev = __shfl_up(key, 1, 64);
  const bool head = lane == 0 || prev != key;
  const uint64_t heads = __ballot(head);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int seg_start = 63 - __clzll(heads & upto);
  const uint64_t after = heads & ~upto;
  const int seg_end = after ? (__ffsll((long long)after) - 2) : 63;
  uint32_t old = 0;
  if (active && lane == seg_end) old = atomicAdd(&acc[key], (uint32_t)(seg_end - seg_start + 1));
  old = __shfl(old, seg_end, 64);
  return old + (uint32_t)(lane - seg_start);
}

// A particle with w == 0 or a cell index outside [0, ncell) is dropped.
__global__ void __launch_bounds__(kSortBlock) k_sort_count(const uint32_t* cell, const uint32_t* w,
                                                          uint32_t n, uint32_t ncell, uint32_t* counts,
                                                          uint32_t* rank) {
  for (uint32_t base = blockIdx.x * blockDim.x; base < n; base += gridDim.x * blockDim.x) {
    const uint32_t i = base + threadIdx.x;
    uint32_t key = kInvalidCell;
    if (i < n && w[i] > 0) {
      const uint32_t c = cell[i];
      key = c < ncell ? c : kInvalidCell;
    }
    const uint32_t r = run_inc(counts, key);
    if (key != kInvalidCell) rank[i] = r;
  }
}

// Exclusive block scan of one value per thread (kSortBlock threads); *total gets the sum.
__device__ __forceinline__ uint32_t sort_block_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  constexpr int nw = kSortBlock / 64;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < nw; ++k) {
    const uint32_t s = sh[k];
    off += k < wid ? s : 0u;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + x - v;
}

__global__ void __launch_bounds__(kSortBlock) k_sort_scan_blocks(const uint32_t* counts, uint32_t ncell,
                                                                uint32_t* part) {
  __shared__ uint32_t sh[kSortBlock / 64];
  const uint32_t nblk = (ncell + kSortTile - 1) / kSortTile;
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    uint32_t v = 0;
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const uint32_t c = b * kSortTile + (uint32_t)j * kSortBlock + threadIdx.x;
      v += c < ncell ? counts[c] : 0u;
    }
    uint32_t tot;
    sort_block_scan(v, sh, &tot);
    if (threadIdx.x == 0) part[b] = tot;
  }
}

// One workgroup: exclusive scan of the block partials in place; part[nblk] = total.
__global__ void __launch_bounds__(kSortTopThreads) k_sort_scan_top(uint32_t* part, uint32_t nblk,
                                                                  uint32_t* n_out) {
  __shared__ uint32_t sh[kSortTopThreads / 64];
  __shared__ uint32_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  const int lane = lane_id(), wid = threadIdx.x >> 6;
  for (uint32_t b0 = 0; b0 < nblk; b0 += kSortTopThreads) {
    const uint32_t b = b0 + threadIdx.x;
    const uint32_t v = b < nblk ? part[b] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t y = __shfl_up(x, d, 64);
      if (lane >= d) x += y;
    }
    if (lane == 63) sh[wid] = x;
    __syncthreads();
    uint32_t off = carry, tot = 0;
    for (int k = 0; k < kSortTopThreads / 64; ++k) {
      const uint32_t s = sh[k];
      off += k < wid ? s : 0u;
      tot += s;
    }
    if (b < nblk) part[b] = off + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[nblk] = carry;
    *n_out = carry;
  }
}

__global__ void __launch_bounds__(kSortBlock) k_sort_scan_down(const uint32_t* counts, uint32_t ncell,
                                                              const uint32_t* part, uint32_t* start) {
  __shared__ uint32_t sh[kSortBlock / 64];
  __shared__ __align__(16) uint32_t tile[kSortTile];
  const uint32_t nblk = (ncell + kSortTile - 1) / kSortTile;
  for (uint32_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const uint32_t cb = b * kSortTile;
    // coalesced loads through LDS, then eight consecutive cells per thread
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const uint32_t i = (uint32_t)j * kSortBlock + threadIdx.x;
      tile[i] = cb + i < ncell ? counts[cb + i] : 0u;
    }
    __syncthreads();
    uint32_t v[kSortPer], s = 0;
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) { v[j] = tile[threadIdx.x * kSortPer + j]; s += v[j]; }
    uint32_t tot;
    uint32_t p = sort_block_scan(s, sh, &tot) + part[b];
#pragma unroll
    for (int j = 0; j < kSortPer; ++j) {
      const uint32_t c = cb + threadIdx.x * kSortPer + (uint32_t)j;
      if (c < ncell) start[c] = p;
      p += v[j];
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) start[ncell] = part[nblk];
}

template <typename T>
__global__ void __launch_bounds__(kSortBlock) k_sort_scatter(const uint32_t* cell, const T* ox, const T* oy,
                                                            const T* oz, const uint32_t* w,
                                                            const uint64_t* id, uint32_t n, uint32_t ncell,
                                                            const uint32_t* start, const uint32_t* rank,
                                                            uint32_t* cell_o, T* ox_o, T* oy_o, T* oz_o,
                                                            uint32_t* w_o, uint64_t* id_o) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t wi = w[i];
    const uint32_t c = cell[i];
    if (wi == 0 || c >= ncell) continue;
    const uint32_t q = start[c] + rank[i];
    cell_o[q] = c;
    ox_o[q] = ox[i];
    oy_o[q] = oy[i];
    oz_o[q] = oz[i];
    w_o[q] = wi;
    id_o[q] = id[i];
  }
}

inline int sort_grid(uint64_t n, uint32_t cap) {
  uint64_t b = (n + kSortBlock - 1) / kSortBlock;
  if (b < 1) b = 1;
  return (int)(b > cap ? cap : b);
}

// The sort on a given scratch of at least sort_words(n, ncell) words.
int sort_run(int precision, uint64_t n, uint32_t ncell, const uint32_t* cell, const void* ox,
             const void* oy, const void* oz, const uint32_t* w, const uint64_t* id, uint32_t* cell_o,
             void* ox_o, void* oy_o, void* oz_o, uint32_t* w_o, uint64_t* id_o, uint32_t* start,
             uint32_t* n_out, uint32_t* scratch, hipStream_t s) {
  auto al = [](uint64_t x) { return (x + 63) & ~(uint64_t)63; };
  uint32_t* counts = scratch;
  uint32_t* rank = counts + al(ncell);
  uint32_t* part = rank + al(n);
  const uint32_t nblk = (ncell + kSortTile - 1) / kSortTile;
  const uint32_t nn = (uint32_t)n;
  // the counters start from zero on every call (a fill kernel, so that a captured call
  // records no memset node)
  k_sort_fill<<<sort_grid(ncell, 2048), kSortBlock, 0, s>>>(counts, ncell);
  if (nn) k_sort_count<<<sort_grid(n, 8192), kSortBlock, 0, s>>>(cell, w, nn, ncell, counts, rank);
  k_sort_scan_blocks<<<nblk < 4096 ? nblk : 4096, kSortBlock, 0, s>>>(counts, ncell, part);
  k_sort_scan_top<<<1, kSortTopThreads, 0, s>>>(part, nblk, n_out);
  k_sort_scan_down<<<nblk < 4096 ? nblk : 4096, kSortBlock, 0, s>>>(counts, ncell, part, start);
  if (nn) {
    if (precision == ITOKMC_FP64)
      k_sort_scatter<double><<<sort_grid(n, 8192), kSortBlock, 0, s>>>(
          cell, (const double*)ox, (const double*)oy, (const double*)oz, w, id, nn, ncell, start, rank, cell_o,
          (double*)ox_o, (double*)oy_o, (double*)oz_o, w_o, id_o);
    else
      k_sort_scatter<float><<<sort_grid(n, 8192), kSortBlock, 0, s>>>(
          cell, (const float*)ox, (const float*)oy, (const float*)oz, w, id, nn, ncell, start, rank, cell_o,
          (float*)ox_o, (float*)oy_o, (float*)oz_o, w_o, id_o);
  }
  return hipGetLastError() == hipSuccess ? ITOKMC_OK : ITOKMC_EHIP;
}

bool sort_args_ok(int precision, uint64_t n, uint32_t ncell, const void* const* p, int np) {
  if (precision != ITOKMC_FP32 && precision != ITOKMC_FP64) return false;
  if (ncell < 1 || ncell > (1u << 24) || n > 0x7FFFFFFFull) return false;
  for (int i = 0; i < np; ++i)
    if (!p[i] && (n > 0 || i >= np - 2)) return false;  // start and n_out always needed
  return true;
}

// ---- file-scope scratch for the no-allocation entry point --------------------------
constexpr uint64_t kNoAllocScratchBytes = 32ull << 20;
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchBytes / 4];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
uint32_t* g_scratch_ptr[kMaxDevices] = {nullptr};

// The device address of this GPU's scratch array, resolved once per device with that
// device current (each GPU holds its own copy at its own address).
hipError_t scratch_for_current_device(uint32_t** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = (uint32_t*)p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace
}  // namespace itk

using namespace itk;

extern "C" {

size_t itokmc_sort_workspace_bytes(uint64_t n, uint32_t ncell) {
  if (ncell < 1 || ncell > (1u << 24) || n > 0x7FFFFFFFull) return 0;
  return (size_t)sort_words(n, ncell) * 4;
}

int itokmc_sort_by_cell(int precision, uint64_t n, uint32_t ncell, const uint32_t* cell, const void* ox,
                        const void* oy, const void* oz, const uint32_t* w, const uint64_t* id,
                        uint32_t* cell_out, void* ox_out, void* oy_out, void* oz_out, uint32_t* w_out,
                        uint64_t* id_out, uint32_t* start, uint32_t* n_out, void* workspace,
                        size_t workspace_bytes, void* stream) {
  const void* p[] = {cell, ox, oy, oz, w, id, cell_out, ox_out, oy_out, oz_out, w_out, id_out, start, n_out};
  if (!sort_args_ok(precision, n, ncell, p, 14) || !workspace) return ITOKMC_EINVAL;
  if (workspace_bytes < (size_t)sort_words(n, ncell) * 4) return ITOKMC_ENOMEM;
  return sort_run(precision, n, ncell, cell, ox, oy, oz, w, id, cell_out, ox_out, oy_out, oz_out, w_out,
                  id_out, start, n_out, (uint32_t*)workspace, (hipStream_t)stream);
}

int itokmc_sort_by_cell_noalloc(int precision, uint64_t n, uint32_t ncell, const uint32_t* cell,
                                const void* ox, const void* oy, const void* oz, const uint32_t* w,
                                const uint64_t* id, uint32_t* cell_out, void* ox_out, void* oy_out,
                                void* oz_out, uint32_t* w_out, uint64_t* id_out, uint32_t* start,
                                uint32_t* n_out, void* stream) {
  const void* p[] = {cell, ox, oy, oz, w, id, cell_out, ox_out, oy_out, oz_out, w_out, id_out, start, n_out};
  if (!sort_args_ok(precision, n, ncell, p, 14)) return ITOKMC_EINVAL;
  if ((uint64_t)sort_words(n, ncell) * 4 > kNoAllocScratchBytes) return ITOKMC_ECAPACITY;
  uint32_t* sp = nullptr;
  if (scratch_for_current_device(&sp) != hipSuccess) return ITOKMC_EHIP;
  return sort_run(precision, n, ncell, cell, ox, oy, oz, w, id, cell_out, ox_out, oy_out, oz_out, w_out,
                  id_out, start, n_out, sp, (hipStream_t)stream);
}

}  // extern "C"
