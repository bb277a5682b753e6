// Device building blocks for gfx950 (wave64): counter-based random numbers and
// wavefront-level aggregation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace itk {

// Philox counter tags (top byte of counter word 3) and particle-id kinds.
enum : uint32_t { TAG_PUSH = 1, TAG_SEED = 2, TAG_KMC = 3, TAG_CREATE = 4, TAG_PHOTON = 5, TAG_ION = 6 };
enum : uint32_t { KIND_SEED = 0, KIND_KMC = 1, KIND_PHOTO = 2, KIND_MERGE = 3 };

constexpr uint32_t kInvalidCell = 0xFFFFFFFFu;

struct Key {
  uint32_t k0, k1;
};

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two 32x32->64
// products of counter words 0 and 2 with fixed multipliers; the key advances by the
// Weyl increments between rounds.
__device__ __forceinline__ uint4 philox(uint4 c, Key key) {
  uint32_t k0 = key.k0, k1 = key.k1;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
    const uint32_t y0 = (uint32_t)(p1 >> 32) ^ c.y ^ k0;
    const uint32_t y2 = (uint32_t)(p0 >> 32) ^ c.w ^ k1;
    c = make_uint4(y0, (uint32_t)p1, y2, (uint32_t)p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

__device__ __forceinline__ uint4 philox_block(uint32_t c0, uint32_t c1, uint32_t c2,
                                              uint32_t tag, uint32_t sub, Key key) {
  return philox(make_uint4(c0, c1, c2, (tag << 24) | (sub & 0xFFFFFFu)), key);
}

// Uniform conversions.  [0,1) at 32-bit resolution, (0,1] at 32-bit resolution (for
// logarithms), and [0,1) at 24-bit resolution (exact in single precision; positions).
__device__ __forceinline__ double u_co(uint32_t x) { return (double)x * 0x1p-32; }
__device__ __forceinline__ double u_oc(uint32_t x) { return ((double)x + 1.0) * 0x1p-32; }
__device__ __forceinline__ double u24(uint32_t x) { return (double)(x >> 8) * 0x1p-24; }
__device__ __forceinline__ float u24f(uint32_t x) { return (float)(x >> 8) * 0x1p-24f; }
// (0,1] in single precision with relative (not absolute) 2^-24 resolution, so that the
// logarithm of small draws stays accurate
__device__ __forceinline__ float u_ocf(uint32_t x) { return __fmaf_rn((float)x, 0x1p-32f, 0x1p-32f); }

// Sequential stream of one cell: word n is word (n mod 4) of the block with counter
// (cell, n div 4, step, tag|sub).
struct CellStream {
  uint32_t cell, step, tagsub;
  Key key;
  uint32_t n;
  uint4 buf;
  __device__ void init(uint32_t c, uint32_t s, uint32_t tag, uint32_t sub, Key k) {
    cell = c; step = s; tagsub = (tag << 24) | sub; key = k; n = 0;
  }
  __device__ __forceinline__ uint32_t next() {
    const uint32_t lane = n & 3u;
    if (lane == 0) buf = philox(make_uint4(cell, n >> 2, step, tagsub), key);
    ++n;
    return lane == 0 ? buf.x : lane == 1 ? buf.y : lane == 2 ? buf.z : buf.w;
  }
};

__device__ __forceinline__ uint64_t make_id(uint32_t kind, uint32_t step, uint32_t cell,
                                            uint32_t slot) {
  return ((uint64_t)kind << 62) | ((uint64_t)(step & 0x3FFFFFu) << 40) |
         ((uint64_t)(cell & 0xFFFFFFu) << 16) | (uint64_t)(slot & 0xFFFFu);
}

// ---- XCD-aware workgroup order --------------------------------------------------
// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.  This
// remaps the dispatch index so XCD x processes one contiguous range of logical blocks:
// neighbouring rows and planes of a stencil then share an L2.  A bijection on
// [0, nblocks).
__device__ __forceinline__ uint32_t xcd_block(uint32_t bid, uint32_t nblocks) {
  const uint32_t per = nblocks >> 3, rem = nblocks & 7u;
  const uint32_t x = bid & 7u, i = bid >> 3;
  return x * per + (x < rem ? x : rem) + i;
}

// ---- wavefront helpers (64 lanes) ------------------------------------------------

// Ordering point between LDS accesses of different lanes inside a workgroup that is one
// wavefront: its lanes run in lockstep and the LDS serves a wavefront's operations in
// issue order, so only the compiler's reordering has to be stopped.  Unlike
// __syncthreads() it does not wait for the wavefront's outstanding global stores.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t shfl_up64(uint64_t v, int d) {
  return (uint64_t)__shfl_up((unsigned long long)v, d, 64);
}
__device__ __forceinline__ uint64_t shfl64(uint64_t v, int src) {
  return (uint64_t)__shfl((unsigned long long)v, src, 64);
}

// Lane moves across the whole wavefront (DPP wave_shr:1 and wave_shl:1): lane i receives
// lane i - 1 (resp. i + 1); the lane with no source receives `fill`.
__device__ __forceinline__ uint32_t dpp_from_prev(uint32_t x, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)x, 0x138, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t dpp_from_next(uint32_t x, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)x, 0x130, 0xF, 0xF, false);
}

// Run-aggregated atomic add.  Lanes whose keys form a run of equal consecutive values
// (inactive lanes use kInvalidCell) add their values to acc[key] with a single atomic
// per run; each active lane receives the value acc[key] had before its own
// contribution (old value plus the exclusive prefix of its run).  Particles sorted by
// cell make runs long, so a wave issues few atomics.
__device__ __forceinline__ uint64_t run_add(unsigned long long* acc, uint32_t key,
                                            uint64_t val) {
  const int lane = lane_id();
  const bool active = key != kInvalidCell;
  const uint32_t prev = dpp_from_prev(key, ~key);
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
  uint64_t old = 0;
  if (active && lane == seg_end) old = atomicAdd(&acc[key], (unsigned long long)x);
  old = shfl64(old, seg_end);
  return old + x - (active ? val : 0ull);
}

// Inclusive prefix sum across the wavefront (32-bit, wrapping) with DPP: shifts by 1,
// 2, 4 and 8 lanes inside each 16-lane row (lanes shifted in from outside the row add
// 0), then the last lane of row 0 added to rows 1 and 3 and the last lane of row 1 (by
// then the total of rows 0-1) to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_prefix_dpp(uint32_t x) {
  x += __builtin_amdgcn_update_dpp(0u, x, 0x111, 0xF, 0xF, true);   // row_shr:1
  x += __builtin_amdgcn_update_dpp(0u, x, 0x112, 0xF, 0xF, true);   // row_shr:2
  x += __builtin_amdgcn_update_dpp(0u, x, 0x114, 0xF, 0xF, true);   // row_shr:4
  x += __builtin_amdgcn_update_dpp(0u, x, 0x118, 0xF, 0xF, true);   // row_shr:8
  x += __builtin_amdgcn_update_dpp(0u, x, 0x142, 0xA, 0xF, false);  // row_bcast:15
  x += __builtin_amdgcn_update_dpp(0u, x, 0x143, 0xC, 0xF, false);  // row_bcast:31
  return x;
}

// One step of a segmented inclusive scan with DPP (control ctrl, rows row_mask): the
// (head flag, value) pair of the source lane combined with the lane's own, keeping the
// lane's value after a head inside its range and applying op otherwise.  The pair
// operator is associative, so the shifts of wave_prefix_dpp (row_shr 1, 2, 4, 8, then
// row_bcast 15 and 31) give the scan of each segment; lanes without a source see the
// identity and no head.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x, uint32_t fill) {
  return (uint32_t)__builtin_amdgcn_update_dpp((int)fill, (int)x, CTRL, ROWS, 0xF, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_u64(uint64_t x, uint64_t fill) {
  const uint32_t lo = dpp_u32<CTRL, ROWS>((uint32_t)x, (uint32_t)fill);
  const uint32_t hi = dpp_u32<CTRL, ROWS>((uint32_t)(x >> 32), (uint32_t)(fill >> 32));
  return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROWS, typename U>
__device__ __forceinline__ U dpp_move(U x, U fill) {
  if constexpr (sizeof(U) == 8) return (U)dpp_u64<CTRL, ROWS>((uint64_t)x, (uint64_t)fill);
  else return (U)dpp_u32<CTRL, ROWS>((uint32_t)x, (uint32_t)fill);
}

// Segmented inclusive scans over the wavefront.  `head` (0/1) marks the first lane of
// a segment; lane 0 always starts one.  Returns the scanned values in place and, in
// `seen`, whether a head lies in lanes 1..i (0: the lane continues lane 0's segment).
template <int CTRL, int ROWS, typename U, int N, typename Op>
__device__ __forceinline__ void seg_step(U (&v)[N], uint32_t& f, const U (&id)[N], Op op) {
  const uint32_t fs = dpp_u32<CTRL, ROWS>(f, 0u);
#pragma unroll
  for (int k = 0; k < N; ++k) {
    const U vs = dpp_move<CTRL, ROWS, U>(v[k], id[k]);
    v[k] = f ? v[k] : op(k, vs, v[k]);
  }
  f |= fs;
}
template <typename U, int N, typename Op>
__device__ __forceinline__ uint32_t seg_scan(U (&v)[N], uint32_t head, const U (&id)[N], Op op) {
  uint32_t f = lane_id() == 0 ? 0u : head;
  seg_step<0x111, 0xF>(v, f, id, op);   // row_shr:1
  seg_step<0x112, 0xF>(v, f, id, op);   // row_shr:2
  seg_step<0x114, 0xF>(v, f, id, op);   // row_shr:4
  seg_step<0x118, 0xF>(v, f, id, op);   // row_shr:8
  seg_step<0x142, 0xA>(v, f, id, op);   // row_bcast:15
  seg_step<0x143, 0xC>(v, f, id, op);   // row_bcast:31
  return f;
}

// The value of one lane (a wave-uniform lane index), read by the scalar unit.
__device__ __forceinline__ uint32_t lane_u32(uint32_t x, int lane) {
  return (uint32_t)__builtin_amdgcn_readlane((int)x, lane);
}
__device__ __forceinline__ uint64_t lane_u64(uint64_t x, int lane) {
  return ((uint64_t)lane_u32((uint32_t)(x >> 32), lane) << 32) | lane_u32((uint32_t)x, lane);
}

// Wavefront sum and maximum with DPP moves (every lane active); the result is uniform.
__device__ __forceinline__ uint64_t wave_sum64_dpp(uint64_t v) {
  uint64_t x[1] = {v};
  const uint64_t id[1] = {0ull};
  (void)seg_scan(x, 0u, id, [](int, uint64_t a, uint64_t b) { return a + b; });
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x[0], 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(x[0] >> 32), 63);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t wave_max_u32_dpp(uint32_t v) {
  uint32_t x[1] = {v};
  const uint32_t id[1] = {0u};
  (void)seg_scan(x, 0u, id, [](int, uint32_t a, uint32_t b) { return a > b ? a : b; });
  return (uint32_t)__builtin_amdgcn_readlane((int)x[0], 63);
}

// Binning of one particle per lane into acc[key] = (count << 32) | weight (inactive
// lanes use kInvalidCell): one 64-bit atomic per run of equal consecutive keys, as
// run_add, but only the count is returned: each active lane's rank in its cell (0 for
// the cell's first particle of the step).  A run's weight is the difference of two
// wavefront prefix sums of 32-bit weights; it is exact because a cell's total weight
// is below 2^32.
__device__ __forceinline__ uint32_t bin_add(unsigned long long* acc, uint32_t key, uint32_t w) {
  const int lane = lane_id();
  const bool active = key != kInvalidCell;
  const uint32_t prev = dpp_from_prev(key, ~key);
  const bool head = (lane == 0) || (prev != key);
  const uint64_t heads = __ballot(head);
  const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int seg_start = 63 - __clzll(heads & upto);
  const uint64_t after = heads & ~upto;
  const int seg_end = after ? (__ffsll((long long)after) - 2) : 63;
  const uint32_t P = wave_prefix_dpp(active ? w : 0u);
  const uint32_t Pb = __shfl(P, seg_start > 0 ? seg_start - 1 : 0, 64);
  const uint32_t wsum = P - (seg_start > 0 ? Pb : 0u);
  uint32_t old = 0;
  if (active && lane == seg_end)
    old = (uint32_t)(atomicAdd(&acc[key], ((unsigned long long)(seg_end - seg_start + 1) << 32) |
                                              (unsigned long long)wsum) >> 32);
  return __shfl(old, seg_end, 64) + (uint32_t)(lane - seg_start);
}

// Scan tiles of 2048 cells.  The binning kernels flag the tile of every cell that
// receives its first particle of the step; the counting-sort scan visits flagged tiles
// only (and clears the flags).
constexpr int kTileShift = 11;
__device__ __forceinline__ void mark_tile(uint32_t* tiles, uint32_t key, uint64_t old) {
  if (key != kInvalidCell && (old >> 32) == 0) {
    uint32_t* f = tiles + (key >> kTileShift);
    // device-coherent read: store only while the tile is still unflagged
    if (__hip_atomic_load(f, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u) *f = 1u;
  }
}

// Wave-wide sum (result valid in every lane).
__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, d, 64);
  return v;
}
__device__ __forceinline__ double wave_sumd(double v) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

// Append n items (per thread) to a counter with one atomic per workgroup; returns the
// thread's first slot.  Every thread of the workgroup must call it (it synchronises);
// sh: 18 words of LDS.
__device__ __forceinline__ uint32_t block_append(uint32_t* counter, uint32_t n, uint32_t* sh) {
  const int lane = lane_id(), wid = threadIdx.x >> 6, nw = (blockDim.x + 63) >> 6;
  uint32_t x = n;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  if (lane == 63) sh[wid] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < nw; ++i) { const uint32_t t = sh[i]; sh[i] = acc; acc += t; }
    sh[17] = acc ? atomicAdd(counter, acc) : 0u;
  }
  __syncthreads();
  const uint32_t r = sh[17] + sh[wid] + x - n;
  __syncthreads();
  return r;
}

// Append n items (per lane) to a counter with one atomic per wave; returns the lane's
// first slot.
__device__ __forceinline__ uint32_t wave_append(uint32_t* counter, uint32_t n) {
  const int lane = lane_id();
  uint32_t x = n;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const uint32_t y = __shfl_up(x, d, 64);
    if (lane >= d) x += y;
  }
  const uint32_t total = __shfl(x, 63, 64);
  uint32_t base = 0;
  if (lane == 63 && total) base = atomicAdd(counter, total);
  base = __shfl(base, 63, 64);
  return base + x - n;
}

}  // namespace itk
