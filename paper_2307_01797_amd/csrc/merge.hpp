// Superparticle merge/split of one cell by one wavefront (section "Superparticle
// management", eq. weight_median).
//
// The cell's live particles (its bank segment plus the slots holding its new KMC
// products) are staged in LDS as pieces (offset, weight, id) in a store addressed
// through two index buffers; a leaf is a contiguous range of an index buffer.  The
// bounding-volume tree grows breadth-first and every leaf of a level is processed at
// once: a leaf splits along the axis of largest extent (single-precision extents, ties
// to the lower axis), its pieces ordered by (coordinate, id); the weight median is the
// first ordered piece p with 2 (weight up to and including p) > leaf weight; a median
// of weight one joins the lighter side (ties left), a heavier median is cut into
// floor(T/2) - W_left (left, omitted if zero) and the rest (right, kept in a spare slot
// at the end of the leaf's region).  Leaves of weight one are terminal; when a level
// would overshoot n_ppc leaves the heaviest split first (ties to the lower index).
// Each final leaf becomes one particle at its weighted centroid with id
// (MERGE, step, cell, leaf).
//
// Leaves are written back into the cell's segment slots, then into its product slots,
// then (splits of small cells only) into slots appended with one atomic; slots left
// over are marked dead (weight 0).
//
// Run by workgroups of exactly one wavefront: the LDS phases are ordered with
// wave_lds_sync(), so the leaf stores of one cell stay in flight while the wavefront
// gathers its next cell.
#pragma once
#include <type_traits>

#include "couple_device.hpp"
#include "device.hpp"
#include "itk.hpp"

namespace itk {

constexpr int kMaxMergePpc = 64;
constexpr int kMergeTiny = 128;   // pieces staged by the common path (smallest LDS)
constexpr int kMergeSmall = 256;  // pieces staged by the mid-size path
template <typename T> struct MergeBig;
template <> struct MergeBig<float> { static constexpr int value = 1536; };
template <> struct MergeBig<double> { static constexpr int value = 1024; };

// Bit pattern whose unsigned order is the order of non-negative values.
template <typename T> struct Bits;
template <> struct Bits<float> {
  using U = uint32_t;
  __device__ static U of(float x) { return __float_as_uint(x); }
  __device__ static float val(U u) { return __uint_as_float(u); }
  static constexpr U lo_init = 0xFFFFFFFFu;
};
template <> struct Bits<double> {
  using U = unsigned long long;
  __device__ static U of(double x) { return (U)__double_as_longlong(x); }
  __device__ static double val(U u) { return __longlong_as_double((long long)u); }
  static constexpr U lo_init = ~0ull;
};

// The small path also stages the sort keys of splitting leaves contiguously.
template <int CAP> struct MergeContig { static constexpr bool value = CAP <= kMergeSmall; };

// In single precision the contiguous path orders pieces by one 64-bit integer: the
// coordinate's bit pattern (ordered like the non-negative value) above the rank of the
// piece's id among the cell's pieces, i.e. by (coordinate, id).
template <typename T, int CAP> struct MergePacked {
  static constexpr bool value = MergeContig<CAP>::value && sizeof(T) == 4;
};

// Index of a store entry in the two index buffers: one byte when the store has at most
// 256 entries (the common staging), else two.
template <int CAP, int NL> struct MergeIdx {
  using type = std::conditional_t<(CAP + NL <= 256), uint8_t, uint16_t>;
};

// NL: leaf capacity (at least n_ppc): 32 for n_ppc <= 32, else kMaxMergePpc.
template <typename T, int CAP, int NL = kMaxMergePpc>
constexpr size_t merge_lds_bytes_c() {
  constexpr size_t S = (size_t)CAP + NL;
  constexpr size_t U = sizeof(typename Bits<T>::U);
  return S * ((MergePacked<T, CAP>::value ? 0 : 8) + 3 * sizeof(T) + 4 +
              2 * sizeof(typename MergeIdx<CAP, NL>::type) + 3)
                            // store (ids in the contiguous array when packed), two index buffers,
                            // three tag arrays
         + (MergeContig<CAP>::value ? S * 8 : 0)               // contiguous ids (packed: keys)
         + (MergeContig<CAP>::value && !MergePacked<T, CAP>::value ? S * sizeof(T) : 0)  // keys
         + (MergePacked<T, CAP>::value ? S * sizeof(typename MergeIdx<CAP, NL>::type) : 0)  // id ranks
         + NL * (2 * 4 + 4 + 6 * U + 1 +                           // weights, extents, axis
                 6 * sizeof(typename MergeIdx<CAP, NL>::type))      // starts, counts, regions,
                                                                    // median positions
         + 64;
}
inline int merge_leaves(int n_ppc) { return n_ppc <= 32 ? 32 : kMaxMergePpc; }

// (coordinate, id rank) as one ordered integer (single precision; -0 folds to +0).
__device__ __forceinline__ uint64_t packed_key(float k, uint32_t r) {
  return ((uint64_t)__float_as_uint(k + 0.0f) << 32) | r;
}
__device__ __forceinline__ uint64_t packed_key(double, uint32_t) { return 0; }


__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Returns 0 if the cell needs no merge, 1 if it was merged, 2 if it holds more than CAP
// pieces (nothing written; the caller defers it to a larger staging area).  gen: the
// cell's M KMC products (weights wb, wb + wr for the first) have not been written to
// their slots [base, base + M) yet; the gather makes them in place (the same values
// write_product stores), and a merged cell's leaves then take those slots directly.
template <typename T, int CAP, int NL>
__device__ int merge_cell(Bank b, Counters* ctr, int which, const StepConst& K, uint32_t c,
                          uint32_t s, uint32_t e, uint32_t base, uint32_t M, int n_ppc,
                          uint64_t* merged, bool gen = false, uint32_t wb = 0, uint32_t wr = 0) {
  using U = typename Bits<T>::U;
  constexpr int S = CAP + NL;
  constexpr uint8_t kNone = 0xFF;
  extern __shared__ __align__(16) char smem[];
  const int lane = lane_id();
  char* p = smem;
  constexpr bool contig = MergeContig<CAP>::value;
  constexpr bool packed = MergePacked<T, CAP>::value;
  // piece ids: needed by the packed path only until the id ranks are known, so there
  // they live in the contiguous key array, which is filled later
  uint64_t* sid_own = (uint64_t*)p; p += packed ? 0 : (size_t)S * 8;
  U* lo = (U*)p; p += (size_t)NL * 3 * sizeof(U);
  U* hi = (U*)p; p += (size_t)NL * 3 * sizeof(U);
  // Arrays selected by a run-time index (axis, buffer) are addressed from one base, so
  // that every access stays an LDS instruction.
  T* const soB = (T*)p; p += (size_t)3 * S * sizeof(T);
  auto so = [soB](int a) { return soB + (size_t)a * S; };
  uint32_t* sw = (uint32_t*)p; p += (size_t)S * 4;
  // leaf records per buffer: weight (u32), start and count (store indices)
  uint32_t* const LWB = (uint32_t*)p; p += (size_t)2 * NL * 4;
  auto LW = [LWB](int k) { return LWB + (size_t)k * NL; };
  uint32_t* medWl = (uint32_t*)p; p += NL * 4;  // weight ordered before the median
  using Ix = typename MergeIdx<CAP, NL>::type;
  Ix* const LSB = (Ix*)p; p += (size_t)4 * NL * sizeof(Ix);
  auto Lst = [LSB](int k) { return LSB + (size_t)k * 2 * NL; };
  auto Lcn = [LSB](int k) { return LSB + (size_t)k * 2 * NL + NL; };
  Ix* Rg = (Ix*)p; p += NL * sizeof(Ix);     // region of each old leaf in the new buffer
  Ix* medp = (Ix*)p; p += NL * sizeof(Ix);   // median position inside the ordered leaf
  Ix* const IB = (Ix*)p; p += (size_t)2 * S * sizeof(Ix);
  auto I = [IB](int k) { return IB + (size_t)k * S; };
  uint8_t* const tagB = (uint8_t*)p; p += (size_t)2 * S;   // leaf of each slot of I(k)
  auto tag = [tagB](int k) { return tagB + (size_t)k * S; };
  uint8_t* otag = (uint8_t*)p; p += (size_t)S;   // splitting leaf owning an ordered slot
  uint8_t* axis = (uint8_t*)p; p += NL;
  p = smem + ((size_t)(p - smem) + 15) / 16 * 16;  // stays an LDS address (LDS instructions)
  uint64_t* kid = (uint64_t*)p; p += contig ? (size_t)S * 8 : 0;   // id (packed: key) of slot q
  uint64_t* const sid = packed ? kid : sid_own;
  T* kkey = (T*)p; p += contig && !packed ? (size_t)S * sizeof(T) : 0;  // key of slot q
  Ix* idr = (Ix*)p; p += packed ? (size_t)S * sizeof(Ix) : 0;   // id rank of store entry

  // ---- gather: segment [s, e) then product slots [base, base + M) ----
  uint32_t m = 0, wmax = 0;
  uint64_t Wtot = 0;
  const uint32_t nseg = e - s;
  for (uint32_t q0 = 0; q0 < nseg + M; q0 += 64) {
    const uint32_t qi = q0 + (uint32_t)lane;
    const uint32_t q = qi < nseg ? s + qi : base + (qi - nseg);
    // product slots past the bank's capacity were never written (overflow is flagged);
    // every word is requested at once (lanes out of range read slot 0, unused)
    const bool inr = qi < nseg + M && q < K.cap;
    const bool made = gen && qi >= nseg;  // a product made here, not read
    const uint32_t qc = inr && !made ? q : 0u;
    uint32_t wq = b.w[qc];
    uint64_t iq = b.id[qc];
    T x0 = reinterpret_cast<const T*>(b.ox)[qc];
    T x1 = reinterpret_cast<const T*>(b.oy)[qc];
    T x2 = reinterpret_cast<const T*>(b.oz)[qc];
    if (made && inr) {
      const Product<T> pr = make_product<T>(c, qi - nseg, wb, wr, K.step, K.key);
      wq = pr.w;
      iq = pr.id;
      x0 = pr.o[0];
      x1 = pr.o[1];
      x2 = pr.o[2];
    }
    const uint32_t w = inr ? wq : 0u;
    const bool alive = w > 0;
    const uint64_t mask = __ballot(alive);
    const uint32_t pos = m + (uint32_t)__popcll(mask & lanemask_lt());
    if (alive) {
      if (pos < (uint32_t)CAP) {
        sid[pos] = iq;
        so(0)[pos] = x0;
        so(1)[pos] = x1;
        so(2)[pos] = x2;
        sw[pos] = w;
        I(0)[pos] = (Ix)pos;
        tag(0)[pos] = 0;
      }
      wmax = w > wmax ? w : wmax;
      Wtot += w;
    }
    m += (uint32_t)__popcll(mask);
  }
  wmax = wave_max_u32_dpp(wmax);
  Wtot = wave_sum64_dpp(Wtot);
  const bool trigger = m > (uint32_t)n_ppc || (m < (uint32_t)n_ppc && wmax >= 2);
  if (!trigger || m == 0) return 0;
  if (m > (uint32_t)CAP) return 2;
  if (lane == 0) { Lst(0)[0] = 0; Lcn(0)[0] = m; LW(0)[0] = (uint32_t)Wtot; }
  wave_lds_sync();
  if (packed) {  // rank of every piece's id among the cell's pieces (ids are distinct here)
    for (uint32_t q = (uint32_t)lane; q < m; q += 64) {
      const uint64_t iq = sid[q];
      uint32_t r = 0, t = 0;
      for (; t + 4 <= m; t += 4)
        r += (sid[t] < iq ? 1u : 0u) + (sid[t + 1] < iq ? 1u : 0u) + (sid[t + 2] < iq ? 1u : 0u) +
             (sid[t + 3] < iq ? 1u : 0u);
      for (; t < m; ++t) r += sid[t] < iq ? 1u : 0u;
      idr[q] = r;
    }
    wave_lds_sync();
  }

  // ---- breadth-first growth, all leaves of a level at once ----
  int cb = 0, nl = 1;
  uint32_t extent = m;   // slots in use in I(cb)
  uint32_t nstore = m;   // next free store entry
  for (int level = 0; level < 64 && nl < n_ppc; ++level) {
    const int ncb = 1 - cb;
    // leaves to split this level
    const uint32_t Wi = lane < nl ? LW(cb)[lane] : 0u;
    const bool cand = lane < nl && Wi >= 2;
    const uint64_t cmask = __ballot(cand);
    const int ncand = __popcll(cmask);
    if (ncand == 0) break;
    const int budget = n_ppc - nl;
    bool chosen = cand;
    if (ncand > budget) {
      int rank = 0;
      for (int j = 0; j < nl; ++j) {
        const uint32_t Wj = lane_u32(Wi, j);
        if (((cmask >> j) & 1ull) && (Wj > Wi || (Wj == Wi && j < lane))) ++rank;
      }
      chosen = cand && rank < budget;
    }
    const uint64_t chm = __ballot(chosen);
    const uint32_t n_i = lane < nl ? Lcn(cb)[lane] : 0u;
    // new leaf index and region of each old leaf (a splitting leaf gets a spare slot)
    const uint32_t widx = lane < nl ? (chosen ? 2u : 1u) : 0u;
    const uint32_t wreg = n_i + (chosen ? 1u : 0u);
    const uint32_t xi = wave_prefix_dpp(widx), xr = wave_prefix_dpp(wreg);
    const uint32_t newidx = xi - widx, R = xr - wreg;
    const int nl_new = (int)lane_u32(xi, 63);
    const uint32_t new_extent = lane_u32(xr, 63);
    if (lane < nl) {
      Rg[lane] = R;
      if (chosen) {
        for (int a = 0; a < 3; ++a) { lo[3 * lane + a] = Bits<T>::lo_init; hi[3 * lane + a] = 0; }
      } else {
        Lst(ncb)[newidx] = R; Lcn(ncb)[newidx] = n_i; LW(ncb)[newidx] = Wi;
      }
    }
    for (uint32_t q = (uint32_t)lane; q < new_extent; q += 64) { tag(ncb)[q] = kNone; otag[q] = kNone; }
    wave_lds_sync();
    // (i) extents of the splitting leaves: a segmented min/max over each 64-slot chunk
    // of the buffer (a leaf's slots are contiguous), then one LDS atomic per leaf
    // segment and bound (LDS atomics of many lanes on one address serialise)
    for (uint32_t q0 = 0; q0 < extent; q0 += 64) {
      const uint32_t q = q0 + (uint32_t)lane;
      const uint8_t L = q < extent ? tag(cb)[q] : kNone;
      const bool part = L != kNone && ((chm >> L) & 1ull);
      const uint32_t key = part ? (uint32_t)L : 0xFFFFFFFFu;
      U mn[3], mx[3];
      if (part) {
        const uint16_t pq = I(cb)[q];
        for (int a = 0; a < 3; ++a) mn[a] = mx[a] = Bits<T>::of(so(a)[pq]);
      } else {
        for (int a = 0; a < 3; ++a) { mn[a] = Bits<T>::lo_init; mx[a] = 0; }
      }
      // segmented min and max of each axis over the chunk (DPP moves, no LDS)
      const uint32_t prev = dpp_from_prev(key, ~key);
      U ext[6] = {mn[0], mn[1], mn[2], mx[0], mx[1], mx[2]};
      const U eid[6] = {Bits<T>::lo_init, Bits<T>::lo_init, Bits<T>::lo_init, 0, 0, 0};
      seg_scan(ext, prev != key ? 1u : 0u, eid,
               [](int k, U a, U b) { return k < 3 ? (a < b ? a : b) : (a > b ? a : b); });
#pragma unroll
      for (int a = 0; a < 3; ++a) { mn[a] = ext[a]; mx[a] = ext[3 + a]; }
      const uint32_t next = dpp_from_next(key, ~key);
      if (part && (lane == 63 || next != key)) {
        for (int a = 0; a < 3; ++a) {
          atomicMin(&lo[3 * L + a], mn[a]);
          atomicMax(&hi[3 * L + a], mx[a]);
        }
      }
    }
    wave_lds_sync();
    if (lane < nl && chosen) {
      float ext[3];
      for (int a = 0; a < 3; ++a)
        ext[a] = (float)((double)Bits<T>::val(hi[3 * lane + a]) - (double)Bits<T>::val(lo[3 * lane + a]));
      int ax = 0;
      if (ext[1] > ext[ax]) ax = 1;
      if (ext[2] > ext[ax]) ax = 2;
      axis[lane] = (uint8_t)ax;
    }
    wave_lds_sync();
    if (contig) {
      for (uint32_t q = (uint32_t)lane; q < extent; q += 64) {
        const uint8_t L = tag(cb)[q];
        if (L == kNone || !((chm >> L) & 1ull)) continue;
        const uint16_t pq = I(cb)[q];
        if (packed) {
          kid[q] = packed_key(so(axis[L])[pq], idr[pq]);
        } else {
          kkey[q] = so(axis[L])[pq];
          kid[q] = sid[pq];
        }
      }
      wave_lds_sync();
    }
    // (ii) order each splitting leaf by (coordinate, id); copy the other leaves
    for (uint32_t q = (uint32_t)lane; q < extent; q += 64) {
      const uint8_t L = tag(cb)[q];
      if (L == kNone) continue;
      const uint32_t Ls = Lst(cb)[L], Ln = Lcn(cb)[L], RL = Rg[L];
      const uint16_t pq = I(cb)[q];
      if (!((chm >> L) & 1ull)) {
        const uint32_t ni = (uint32_t)L + (uint32_t)__popcll(chm & ((1ull << L) - 1ull));
        I(ncb)[RL + (q - Ls)] = (Ix)pq;
        tag(ncb)[RL + (q - Ls)] = (uint8_t)ni;
        continue;
      }
      const int ax = axis[L];
      const T kq = so(ax)[pq];
      const uint64_t iq = packed ? 0ull : sid[pq];
      uint32_t rank = 0;
      if (packed) {
        const uint64_t cq = packed_key(kq, idr[pq]);
        uint32_t r = Ls;
        const uint32_t rend = Ls + Ln;
        for (; r + 4 <= rend; r += 4)
          rank += (kid[r] < cq ? 1u : 0u) + (kid[r + 1] < cq ? 1u : 0u) + (kid[r + 2] < cq ? 1u : 0u) +
                  (kid[r + 3] < cq ? 1u : 0u);
        for (; r < rend; ++r) rank += kid[r] < cq ? 1u : 0u;
      } else if (contig) {
        uint32_t r = Ls;
        const uint32_t rend = Ls + Ln;
        for (; r + 4 <= rend; r += 4) {
          const T k0 = kkey[r], k1 = kkey[r + 1], k2 = kkey[r + 2], k3 = kkey[r + 3];
          const uint64_t i0 = kid[r], i1 = kid[r + 1], i2 = kid[r + 2], i3 = kid[r + 3];
          rank += (k0 < kq || (k0 == kq && i0 < iq)) ? 1u : 0u;
          rank += (k1 < kq || (k1 == kq && i1 < iq)) ? 1u : 0u;
          rank += (k2 < kq || (k2 == kq && i2 < iq)) ? 1u : 0u;
          rank += (k3 < kq || (k3 == kq && i3 < iq)) ? 1u : 0u;
        }
        for (; r < rend; ++r) {
          const T kr = kkey[r];
          rank += (kr < kq || (kr == kq && kid[r] < iq)) ? 1u : 0u;
        }
      } else {
        for (uint32_t r = Ls; r < Ls + Ln; ++r) {
          const uint16_t pr = I(cb)[r];
          const T kr = so(ax)[pr];
          rank += (kr < kq || (kr == kq && sid[pr] < iq)) ? 1u : 0u;
        }
      }
      I(ncb)[RL + rank] = (Ix)pq;
      otag[RL + rank] = L;
    }
    wave_lds_sync();
    // (iii) weight median of every splitting leaf: one segmented scan over the buffer.
    // A leaf's weight is below 2^32 (LW), so its prefix sums are exact in 32 bits.  The
    // pieces of a leaf all weigh at least 1, so its prefix x rises strictly: a slot
    // lies left of the median if 2x <= W, right of it if 2(x - w) > W, and is the
    // median otherwise; the first two get their child's tag here, the median (and a
    // split superparticle's spare slot) with the children below.
    uint32_t carry = 0;
    uint32_t carry_key = 0xFFFFFFFFu;
    bool carry_hit = false;
    for (uint32_t q0 = 0; q0 < new_extent; q0 += 64) {
      const uint32_t q = q0 + (uint32_t)lane;
      const uint8_t t8 = q < new_extent ? otag[q] : kNone;
      const bool valid = t8 != kNone;
      const uint32_t vkey = valid ? (uint32_t)t8 : 0xFFFFFFFFu;
      const uint32_t w = valid ? sw[I(ncb)[q]] : 0u;
      // segmented prefix sums of the weights over the chunk (DPP moves, no LDS)
      const uint32_t prev = dpp_from_prev(vkey, ~vkey);
      uint32_t xs[1] = {w};
      const uint32_t zid[1] = {0u};
      const uint32_t seen = seg_scan(xs, prev != vkey ? 1u : 0u, zid,
                                     [](int, uint32_t a, uint32_t b) { return a + b; });
      uint32_t x = xs[0];
      if (!seen && vkey == carry_key) x += carry;
      const uint32_t Wv = valid ? LW(cb)[vkey & 63u] : 0u;
      const bool hit = valid && x > Wv - x;  // 2x > W
      const bool up_hit = dpp_from_prev(hit ? 1u : 0u, 0u) != 0u;
      const bool prev_same = lane > 0 ? prev == vkey : vkey == carry_key;
      const bool prev_hit = lane > 0 ? up_hit : carry_hit;
      if (hit && !(prev_same && prev_hit)) {
        medp[vkey] = q - Rg[vkey];
        medWl[vkey] = x - w;
      }
      if (valid) {
        const uint32_t ni = vkey + (uint32_t)__popcll(chm & ((1ull << vkey) - 1ull));
        const uint32_t xe = x - w;
        tag(ncb)[q] = !hit ? (uint8_t)ni : (xe > Wv - xe ? (uint8_t)(ni + 1u) : kNone);
      }
      carry = lane_u32(x, 63);
      carry_key = lane_u32(vkey, 63);
      carry_hit = lane_u32(hit ? 1u : 0u, 63) != 0u;
    }
    wave_lds_sync();
    // (iv)-(v) children of every splitting leaf, one lane per leaf
    uint32_t lcnt = 0, rst = 0, rcnt = 0, WLn = 0, WRn = 0, wl = 0, pm = 0, mu = 0;
    bool super = false;
    if (lane < nl && chosen) {
      mu = medp[lane];
      const uint32_t Wl = medWl[lane];
      pm = I(ncb)[R + mu];
      const uint32_t wm = sw[pm];
      const uint32_t Wr = Wi - Wl - wm;
      if (wm == 1) {
        if (Wl <= Wr) { lcnt = mu + 1; rst = mu + 1; rcnt = n_i - mu - 1; WLn = Wl + 1; WRn = Wr; }
        else { lcnt = mu; rst = mu; rcnt = n_i - mu; WLn = Wl; WRn = Wr + 1; }
      } else {
        super = true;
        wl = (Wl + wm + Wr) / 2 - Wl;
        lcnt = wl > 0 ? mu + 1 : mu;
        rst = mu + 1; rcnt = n_i - mu;
        WLn = Wl + wl; WRn = Wr + (wm - wl);
      }
    }
    // store entries for the right pieces of split superparticle medians
    const uint32_t sx = super ? 1u : 0u;
    const uint32_t sp = wave_prefix_dpp(sx);
    const uint32_t np = nstore + sp - sx;
    nstore += lane_u32(sp, 63);
    if (lane < nl && chosen) {
      if (super) {
        const uint32_t wm = sw[pm];
        if (packed) idr[np] = idr[pm];
        else sid[np] = sid[pm];
        for (int a = 0; a < 3; ++a) so(a)[np] = so(a)[pm];
        sw[np] = wm - wl;
        sw[pm] = wl;
        I(ncb)[R + n_i] = (Ix)np;
      }
      Lst(ncb)[newidx] = R; Lcn(ncb)[newidx] = lcnt; LW(ncb)[newidx] = WLn;
      Lst(ncb)[newidx + 1] = R + rst; Lcn(ncb)[newidx + 1] = rcnt; LW(ncb)[newidx + 1] = WRn;
      // the median slot joins the left child if the left count covers it, else the
      // right one (a unit median) or none (a split superparticle whose left part is
      // empty); a split superparticle's right part, in the spare slot, closes the
      // right child
      tag(ncb)[R + mu] = lcnt > mu ? (uint8_t)newidx : (super ? kNone : (uint8_t)(newidx + 1u));
      if (super) tag(ncb)[R + n_i] = (uint8_t)(newidx + 1u);
    }
    wave_lds_sync();
    cb = ncb;
    nl = nl_new;
    extent = new_extent;
  }

  // ---- leaves -> particles ----
  double my_o[3] = {0.0, 0.0, 0.0};
  uint32_t my_w = 0;
  if (lane < nl) {
    const uint32_t st = Lst(cb)[lane], n = Lcn(cb)[lane];
    double acc[3] = {0.0, 0.0, 0.0};
    for (uint32_t q = st; q < st + n; ++q) {
      const uint16_t pq = I(cb)[q];
      const double w = (double)sw[pq];
      for (int a = 0; a < 3; ++a) acc[a] += w * (double)so(a)[pq];
    }
    my_w = LW(cb)[lane];
    for (int a = 0; a < 3; ++a) my_o[a] = acc[a] / (double)my_w;
  }
  uint32_t extra_base = 0;
  const int extra = nl - (int)nseg - (int)M;
  if (extra > 0) {
    if (lane == 0) extra_base = atomicAdd(&ctr->n[which], (uint32_t)extra);
    extra_base = lane_u32(extra_base, 0);
  }
  if (lane < nl) {
    const uint32_t i = (uint32_t)lane;
    uint32_t q;
    if (i < nseg) q = s + i;
    else if (i < nseg + M) q = base + (i - nseg);
    else q = extra_base + (i - nseg - M);
    if (q < K.cap) {
      T o3[3];
      for (int a = 0; a < 3; ++a) {
        double v = my_o[a];
        v = v < 0.0 ? 0.0 : v;
        T t = (T)v;
        if (!(t < (T)1)) t = sizeof(T) == 4 ? (T)0x1.fffffep-1f : (T)0x1.fffffffffffffp-1;
        o3[a] = t;
      }
      b.cell[q] = c;
      reinterpret_cast<T*>(b.ox)[q] = o3[0];
      reinterpret_cast<T*>(b.oy)[q] = o3[1];
      reinterpret_cast<T*>(b.oz)[q] = o3[2];
      b.w[q] = my_w;
      b.id[q] = make_id(KIND_MERGE, K.step, c, i);
    } else {
      atomicOr(&ctr->overflow, 1u);
    }
  }
  // retire the cell's remaining slots
  for (uint32_t i = (uint32_t)nl + (uint32_t)lane; i < nseg + M; i += 64) {
    const uint32_t q = i < nseg ? s + i : base + (i - nseg);
    if (q < K.cap) b.w[q] = 0;
  }
  if (lane == 0) *merged += 1;
  wave_lds_sync();
  return 1;
}

}  // namespace itk
