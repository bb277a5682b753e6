// Superparticle merge/split of one cell by one wavefront (section "Superparticle
// management", eq. weight_median).
//
// The cell's live particles plus its new KMC products are staged in LDS as pieces
// (offset, weight, id).  A bounding-volume tree is grown breadth-first: a leaf splits
// along the axis of largest extent (single-precision extents, ties to the lower
// axis), its pieces ordered by (coordinate, id); the weight median is the first sorted
// piece p with 2 (weight up to and including p) > leaf weight; a median of weight one
// joins the lighter side (ties left), a heavier median is cut into floor(T/2) - W_left
// (left, omitted if zero) and the rest (right).  Leaves of weight one are terminal;
// when a level would overshoot n_ppc leaves the heaviest split first (ties to the
// lower index).  Each final leaf becomes one particle at its weighted centroid with
// id (MERGE, step, cell, leaf).
//
// Leaves are written back into the cell's own bank slots, then into the slots the KMC
// pass reserved for the products, then (splits of small cells only) into slots
// appended with one atomic; slots left over are marked dead (weight 0).
#pragma once
#include "device.hpp"
#include "itk.hpp"

namespace itk {

template <typename T> struct MergeCap;
template <> struct MergeCap<float> { static constexpr int value = 1536; };
template <> struct MergeCap<double> { static constexpr int value = 1024; };
constexpr int kMaxMergePpc = 64;

struct MergeScratch {
  int n_ppc;
};

inline MergeScratch merge_scratch(itokmc_ctx* ctx) { return MergeScratch{ctx->d.n_ppc}; }

template <typename T>
inline size_t merge_lds_bytes(int n_ppc) {
  if (n_ppc <= 0) return 0;
  const size_t cap2 = (size_t)MergeCap<T>::value + (size_t)n_ppc;
  return cap2 * (8 + 3 * sizeof(T) + 4) + 2 * cap2 * 2 + 2 * 3 * 4 * (size_t)kMaxMergePpc + 64;
}

// Piece store (each piece once) plus two index buffers whose ranges are the leaves.
template <typename T>
struct Pieces {
  uint64_t* id;
  T* o[3];
  uint32_t* w;
};

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

template <typename T>
__device__ bool merge_cell(Bank b, Counters* ctr, int which, const StepConst& K, uint32_t c,
                           uint32_t s, uint32_t e, uint32_t M, uint32_t base, const T no[3],
                           uint32_t nw, uint64_t nid, int n_ppc, const MergeScratch&,
                           uint64_t* merged) {
  extern __shared__ __align__(16) char smem[];
  constexpr int CAP = MergeCap<T>::value;
  const int cap2 = CAP + n_ppc;
  const int lane = lane_id();
  Pieces<T> S;
  char* p = smem;
  S.id = (uint64_t*)p; p += (size_t)cap2 * 8;
  for (int a = 0; a < 3; ++a) { S.o[a] = (T*)p; p += (size_t)cap2 * sizeof(T); }
  S.w = (uint32_t*)p; p += (size_t)cap2 * 4;
  uint16_t* I[2];
  for (int k = 0; k < 2; ++k) { I[k] = (uint16_t*)p; p += (size_t)cap2 * 2; }
  uint32_t* Lst[2];
  uint32_t* Lcn[2];
  uint32_t* LW[2];
  for (int k = 0; k < 2; ++k) {
    Lst[k] = (uint32_t*)p; p += kMaxMergePpc * 4;
    Lcn[k] = (uint32_t*)p; p += kMaxMergePpc * 4;
    LW[k] = (uint32_t*)p; p += kMaxMergePpc * 4;
  }

  // ---- gather live particles and the new products ----
  uint32_t m = 0, wmax = 0;
  uint64_t Wtot = 0;
  for (uint32_t q0 = s; q0 < e; q0 += 64) {
    const uint32_t q = q0 + (uint32_t)lane;
    const uint32_t w = q < e ? b.w[q] : 0u;
    const bool alive = w > 0;
    const uint64_t mask = __ballot(alive);
    const uint32_t pos = m + (uint32_t)__popcll(mask & lanemask_lt());
    if (alive) {
      if (pos < (uint32_t)CAP) {
        S.id[pos] = b.id[q];
        S.o[0][pos] = reinterpret_cast<const T*>(b.ox)[q];
        S.o[1][pos] = reinterpret_cast<const T*>(b.oy)[q];
        S.o[2][pos] = reinterpret_cast<const T*>(b.oz)[q];
        S.w[pos] = w;
        I[0][pos] = (uint16_t)pos;
      }
      wmax = w > wmax ? w : wmax;
      Wtot += w;
    }
    m += (uint32_t)__popcll(mask);
  }
  if ((uint32_t)lane < M) {
    const uint32_t pos = m + (uint32_t)lane;
    if (pos < (uint32_t)CAP) {
      S.id[pos] = nid;
      S.o[0][pos] = no[0];
      S.o[1][pos] = no[1];
      S.o[2][pos] = no[2];
      S.w[pos] = nw;
      I[0][pos] = (uint16_t)pos;
    }
    wmax = nw > wmax ? nw : wmax;
    Wtot += nw;
  }
  m += M;
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint32_t o = __shfl_xor(wmax, d, 64);
    wmax = o > wmax ? o : wmax;
  }
  Wtot = wave_sum64(Wtot);
  const bool trigger = m > (uint32_t)n_ppc || (m < (uint32_t)n_ppc && wmax >= 2);
  if (!trigger || m == 0) return false;
  if (m > (uint32_t)CAP) {
    if (lane == 0) atomicAdd(&ctr->merge_skipped, 1u);
    return false;
  }
  __syncthreads();

  // ---- breadth-first tree growth ----
  int cb = 0, cl = 0, nl = 1;
  uint32_t nstore = m;  // next free piece in the store (split superparticle pieces)
  if (lane == 0) { Lst[0][0] = 0; Lcn[0][0] = m; LW[0][0] = (uint32_t)Wtot; }
  __syncthreads();
  for (int level = 0; level < 64 && nl < n_ppc; ++level) {
    const uint32_t Wi = lane < nl ? LW[cl][lane] : 0u;
    const bool cand = lane < nl && Wi >= 2;
    const uint64_t cmask = __ballot(cand);
    const int ncand = __popcll(cmask);
    if (ncand == 0) break;
    const int budget = n_ppc - nl;
    bool chosen = cand;
    if (ncand > budget) {
      int rank = 0;
      for (int j = 0; j < nl; ++j) {
        const uint32_t Wj = __shfl(Wi, j, 64);
        const bool cj = (cmask >> j) & 1ull;
        if (cj && (Wj > Wi || (Wj == Wi && j < lane))) ++rank;
      }
      chosen = cand && rank < budget;
    }
    const uint64_t chmask = __ballot(chosen);
    // new leaf index and new piece-region start of each old leaf
    const uint32_t cnt_i = lane < nl ? Lcn[cl][lane] : 0u;
    uint32_t widx = lane < nl ? (chosen ? 2u : 1u) : 0u;
    uint32_t wreg = cnt_i + (chosen ? 1u : 0u);
    uint32_t xi = widx, xr = wreg;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint32_t yi = __shfl_up(xi, d, 64), yr = __shfl_up(xr, d, 64);
      if (lane >= d) { xi += yi; xr += yr; }
    }
    const uint32_t newidx = xi - widx, region = xr - wreg;
    const int nl_new = (int)__shfl(xi, 63, 64);
    const int ncb = 1 - cb, ncl = 1 - cl;
    for (int L = 0; L < nl; ++L) {
      const uint32_t st = Lst[cl][L], n = Lcn[cl][L], WL = LW[cl][L];
      const uint32_t R = __shfl(region, L, 64), ni = __shfl(newidx, L, 64);
      if (!((chmask >> L) & 1ull)) {
        for (uint32_t q = (uint32_t)lane; q < n; q += 64) I[ncb][R + q] = I[cb][st + q];
        if (lane == 0) { Lst[ncl][ni] = R; Lcn[ncl][ni] = n; LW[ncl][ni] = WL; }
        continue;
      }
      // (i) axis of largest extent
      T lo[3], hi[3];
      for (int a = 0; a < 3; ++a) { lo[a] = S.o[a][I[cb][st]]; hi[a] = lo[a]; }
      for (uint32_t q = (uint32_t)lane; q < n; q += 64)
        for (int a = 0; a < 3; ++a) {
          const T v = S.o[a][I[cb][st + q]];
          lo[a] = v < lo[a] ? v : lo[a];
          hi[a] = v > hi[a] ? v : hi[a];
        }
      float ext[3];
      for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
          const T ol = __shfl_xor(lo[a], d, 64), oh = __shfl_xor(hi[a], d, 64);
          lo[a] = ol < lo[a] ? ol : lo[a];
          hi[a] = oh > hi[a] ? oh : hi[a];
        }
        ext[a] = (float)((double)hi[a] - (double)lo[a]);
      }
      int ax = 0;
      if (ext[1] > ext[ax]) ax = 1;
      if (ext[2] > ext[ax]) ax = 2;
      // (ii) order by (coordinate, id): rank of each piece, written to the new region
      for (uint32_t q = (uint32_t)lane; q < n; q += 64) {
        const uint16_t pq = I[cb][st + q];
        const T kq = S.o[ax][pq];
        const uint64_t iq = S.id[pq];
        uint32_t rank = 0;
        for (uint32_t r = 0; r < n; ++r) {
          const uint16_t pr = I[cb][st + r];
          const T kr = S.o[ax][pr];
          const uint64_t ir = S.id[pr];
          rank += (kr < kq || (kr == kq && ir < iq)) ? 1u : 0u;
        }
        I[ncb][R + rank] = pq;
      }
      __syncthreads();
      // (iii) weight median: first sorted piece with 2 * inclusive weight > leaf weight
      uint64_t run = 0;
      int med = -1;
      uint64_t Wl = 0;
      for (uint32_t q0 = 0; q0 < n && med < 0; q0 += 64) {
        const uint32_t q = q0 + (uint32_t)lane;
        const uint64_t w = q < n ? (uint64_t)S.w[I[ncb][R + q]] : 0ull;
        uint64_t x = w;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint64_t y = shfl_up64(x, d);
          if (lane >= d) x += y;
        }
        const bool hit = q < n && 2ull * (run + x) > (uint64_t)WL;
        const uint64_t hm = __ballot(hit);
        if (hm) {
          const int first = __ffsll((long long)hm) - 1;
          med = (int)q0 + first;
          Wl = run + shfl64(x - w, first);
        }
        run += shfl64(x, 63);
      }
      const uint32_t mu = (uint32_t)med;
      const uint16_t pm = I[ncb][R + mu];
      const uint32_t wm = S.w[pm];
      const uint64_t Wr = (uint64_t)WL - Wl - wm;
      // (iv)-(v) children.  The region holds n + 1 slots: a split superparticle median
      // keeps its left piece in place and puts its right piece in the spare last slot.
      uint32_t lcnt, rst, rcnt;
      uint64_t WLn, WRn;
      if (wm == 1) {
        if (Wl <= Wr) {  // median joins the left side
          lcnt = mu + 1; rst = mu + 1; rcnt = n - mu - 1;
          WLn = Wl + 1; WRn = Wr;
        } else {         // median joins the right side
          lcnt = mu; rst = mu; rcnt = n - mu;
          WLn = Wl; WRn = Wr + 1;
        }
      } else {
        const uint64_t Ttot = Wl + wm + Wr;
        const uint32_t wl = (uint32_t)(Ttot / 2 - Wl);
        const uint32_t wr = wm - wl;
        if (lane == 0) {
          const uint32_t np = nstore;
          S.id[np] = S.id[pm];
          for (int a = 0; a < 3; ++a) S.o[a][np] = S.o[a][pm];
          S.w[np] = wr;
          S.w[pm] = wl;
          I[ncb][R + n] = (uint16_t)np;
        }
        ++nstore;
        lcnt = wl > 0 ? mu + 1 : mu;
        rst = mu + 1; rcnt = n - mu;
        WLn = Wl + wl; WRn = Wr + wr;
      }
      if (lane == 0) {
        Lst[ncl][ni] = R; Lcn[ncl][ni] = lcnt; LW[ncl][ni] = (uint32_t)WLn;
        Lst[ncl][ni + 1] = R + rst; Lcn[ncl][ni + 1] = rcnt; LW[ncl][ni + 1] = (uint32_t)WRn;
      }
      __syncthreads();
    }
    __syncthreads();
    cb = ncb;
    cl = ncl;
    nl = nl_new;
  }

  // ---- leaves -> particles ----
  double my_o[3] = {0.0, 0.0, 0.0};
  uint32_t my_w = 0;
  for (int L = 0; L < nl; ++L) {
    const uint32_t st = Lst[cl][L], n = Lcn[cl][L];
    double acc[3] = {0.0, 0.0, 0.0};
    for (uint32_t q = (uint32_t)lane; q < n; q += 64) {
      const uint16_t pq = I[cb][st + q];
      const double w = (double)S.w[pq];
      for (int a = 0; a < 3; ++a) acc[a] += w * (double)S.o[a][pq];
    }
    for (int a = 0; a < 3; ++a) acc[a] = wave_sumd(acc[a]);
    if (lane == L) {
      my_w = LW[cl][L];
      for (int a = 0; a < 3; ++a) my_o[a] = acc[a] / (double)my_w;
    }
  }
  const uint32_t seg_n = e - s;
  uint32_t extra_base = 0;
  const int extra = nl - (int)seg_n - (int)M;
  if (extra > 0) {
    if (lane == 0) extra_base = atomicAdd(&ctr->n[which], (uint32_t)extra);
    extra_base = __shfl(extra_base, 0, 64);
  }
  if (lane < nl) {
    uint32_t q;
    const uint32_t i = (uint32_t)lane;
    if (i < seg_n) q = s + i;
    else if (i < seg_n + M) q = base + (i - seg_n);
    else q = extra_base + (i - seg_n - M);
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
  for (uint32_t i = (uint32_t)nl + (uint32_t)lane; i < seg_n; i += 64) b.w[s + i] = 0;
  const uint32_t used_res = nl > (int)seg_n ? (uint32_t)(nl - (int)seg_n) : 0u;
  for (uint32_t i = used_res + (uint32_t)lane; i < M; i += 64) {
    const uint32_t q = base + i;
    if (q < K.cap) b.w[q] = 0;
  }
  if (lane == 0) *merged += 1;
  __syncthreads();
  return true;
}

}  // namespace itk
