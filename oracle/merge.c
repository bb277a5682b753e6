/*
 * Oracle: superparticle merge/split of one cell (test infrastructure; see oracle.h).
 *
 * Follows the paper's section "Superparticle management": a bounding-volume tree is
 * grown top-down; a leaf is split by (i) taking the axis of largest bounding-box
 * extent, (ii) sorting along it, (iii) locating the weight median p' of eq.
 * weight_median, (iv) sending p < p' left and p > p' right, and (v) giving a physical
 * median particle to the lighter side or splitting a superparticle median so the two
 * sides differ by at most one.  Growth stops at N_ppc leaves; each leaf becomes one
 * particle with the summed weight at the weighted centroid (eqs. for w and X at the
 * end of that section).
 *
 * Readings where the text is silent or ambiguous:
 *   - "p' > 1" is read as p' >= 1 (1-based), i.e. the first index may be the median;
 *   - extents are compared as single-precision differences of the cell-relative
 *     offsets, ties going to the lowest axis; the sort key is (coordinate, id);
 *   - a physical median joins the lighter side, a tie going left; a superparticle
 *     median of weight w is cut into floor(T/2) - W_l (left, omitted when zero) and
 *     the rest (right), T = W_l + w + W_r;
 *   - growth is breadth-first: a leaf of total weight 1 is terminal; when a level
 *     would overshoot N_ppc the heaviest leaves split first, ties to the lower index;
 *   - every leaf gets a new id (MERGE, step, cell, leaf index) and its offset is
 *     clamped into [0,1).
 * Pins (tests): the paper's example (1000 particles, weights uniform in 1..100,
 * merged to 64 leaves whose weights differ by at most one); the split of a single
 * superparticle; weight and centroid conservation; brute-force median on tiny sets.
 */
#include "or_internal.h"

typedef struct {
  double o[3];
  uint64_t w;
  uint64_t id;
} piece;

typedef struct {
  piece* p;
  int32_t n;
  uint64_t W;
} leaf;

static int g_axis; /* sort axis for qsort */
static int cmp_piece(const void* a, const void* b) {
  const piece* x = (const piece*)a;
  const piece* y = (const piece*)b;
  if (x->o[g_axis] < y->o[g_axis]) return -1;
  if (x->o[g_axis] > y->o[g_axis]) return 1;
  return (x->id < y->id) ? -1 : (x->id > y->id) ? 1 : 0;
}

static void split_leaf(const leaf* L, leaf* left, leaf* right) {
  /* (i) axis of largest extent */
  float ext[3];
  for (int a = 0; a < 3; ++a) {
    double lo = L->p[0].o[a], hi = L->p[0].o[a];
    for (int i = 1; i < L->n; ++i) {
      if (L->p[i].o[a] < lo) lo = L->p[i].o[a];
      if (L->p[i].o[a] > hi) hi = L->p[i].o[a];
    }
    ext[a] = (float)(hi - lo);
  }
  int axis = 0;
  if (ext[1] > ext[axis]) axis = 1;
  if (ext[2] > ext[axis]) axis = 2;
  /* (ii) sort */
  piece* q = (piece*)malloc(sizeof(piece) * (size_t)L->n);
  memcpy(q, L->p, sizeof(piece) * (size_t)L->n);
  g_axis = axis;
  qsort(q, (size_t)L->n, sizeof(piece), cmp_piece);
  /* (iii) weight median: smallest m (0-based) with sum_{p<m} w + w_m > sum_{p>m} w */
  uint64_t total = 0;
  for (int i = 0; i < L->n; ++i) total += q[i].w;
  uint64_t below = 0;
  int m = 0;
  for (m = 0; m < L->n; ++m) {
    uint64_t above = total - below - q[m].w;
    if (below + q[m].w > above) break;
    below += q[m].w;
  }
  uint64_t Wl = below, Wr = total - below - q[m].w;
  /* (iv) */
  left->p = (piece*)malloc(sizeof(piece) * (size_t)(L->n + 1));
  right->p = (piece*)malloc(sizeof(piece) * (size_t)(L->n + 1));
  left->n = right->n = 0;
  for (int i = 0; i < m; ++i) left->p[left->n++] = q[i];
  for (int i = m + 1; i < L->n; ++i) right->p[right->n++] = q[i];
  /* (v) median */
  piece med = q[m];
  if (med.w == 1) {
    if (Wl <= Wr) { left->p[left->n++] = med; Wl += 1; }
    else { right->p[right->n++] = med; Wr += 1; }
  } else {
    uint64_t T = Wl + med.w + Wr;
    uint64_t wl = T / 2 - Wl;
    uint64_t wr = med.w - wl;
    if (wl > 0) { piece a = med; a.w = wl; left->p[left->n++] = a; Wl += wl; }
    piece b = med; b.w = wr; right->p[right->n++] = b; Wr += wr;
  }
  left->W = Wl;
  right->W = Wr;
  free(q);
}

int32_t or_merge_cell(int32_t n_ppc, int32_t m, const double* off, const uint64_t* w,
                      const uint64_t* id, uint32_t cell, uint32_t step, double* out_off,
                      uint64_t* out_w, uint64_t* out_id) {
  if (m <= 0 || n_ppc <= 0) return 0;
  leaf* leaves = (leaf*)malloc(sizeof(leaf) * (size_t)n_ppc);
  leaf* next = (leaf*)malloc(sizeof(leaf) * (size_t)n_ppc);
  int32_t nl = 1;
  leaves[0].n = m;
  leaves[0].p = (piece*)malloc(sizeof(piece) * (size_t)m);
  leaves[0].W = 0;
  for (int i = 0; i < m; ++i) {
    for (int a = 0; a < 3; ++a) leaves[0].p[i].o[a] = off[3 * i + a];
    leaves[0].p[i].w = w[i];
    leaves[0].p[i].id = id[i];
    leaves[0].W += w[i];
  }
  for (;;) {
    if (nl >= n_ppc) break;
    int32_t ncand = 0;
    for (int i = 0; i < nl; ++i) if (leaves[i].W >= 2) ncand++;
    if (ncand == 0) break;
    int32_t budget = n_ppc - nl;
    char* chosen = (char*)calloc((size_t)nl, 1);
    if (ncand <= budget) {
      for (int i = 0; i < nl; ++i) chosen[i] = leaves[i].W >= 2;
    } else {
      /* pick the `budget` heaviest splittable leaves, ties to the lower index */
      for (int k = 0; k < budget; ++k) {
        int best = -1;
        for (int i = 0; i < nl; ++i) {
          if (chosen[i] || leaves[i].W < 2) continue;
          if (best < 0 || leaves[i].W > leaves[best].W) best = i;
        }
        chosen[best] = 1;
      }
    }
    int32_t nn = 0;
    for (int i = 0; i < nl; ++i) {
      if (chosen[i]) {
        split_leaf(&leaves[i], &next[nn], &next[nn + 1]);
        free(leaves[i].p);
        nn += 2;
      } else {
        next[nn++] = leaves[i];
      }
    }
    free(chosen);
    leaf* t = leaves; leaves = next; next = t;
    nl = nn;
  }
  for (int i = 0; i < nl; ++i) {
    double acc[3] = {0, 0, 0};
    uint64_t W = 0;
    for (int j = 0; j < leaves[i].n; ++j) {
      for (int a = 0; a < 3; ++a) acc[a] += (double)leaves[i].p[j].w * leaves[i].p[j].o[a];
      W += leaves[i].p[j].w;
    }
    for (int a = 0; a < 3; ++a) {
      double o = acc[a] / (double)W;
      if (o < 0.0) o = 0.0;
      if (o >= 1.0) o = nextafter(1.0, 0.0);
      out_off[3 * i + a] = o;
    }
    out_w[i] = W;
    out_id[i] = or_make_id(OR_KIND_MERGE, step, cell, (uint32_t)i);
    free(leaves[i].p);
  }
  free(leaves);
  free(next);
  return nl;
}
