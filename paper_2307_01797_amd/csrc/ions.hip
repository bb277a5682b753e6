// Mobile ions on the grid.  The paper moves ions as Ito particles (positive ions along
// E, eq. Vk1 with sgn(Z) = +1) and proposes heavy species as a continuum in its
// future-work section.  Here the ions stay the per-cell integer counts of the reaction
// network and move as a lattice jump process, the first-order upwind finite-volume
// form of the drift-diffusion equation realised with integer jumps: an ion of sign q
// crosses the face towards its neighbour along axis a in direction d (-1, +1) at the rate
//     max(0, d q mu_ion E_face,a) / dx + D_ion / dx^2,
// E_face the mean of the two cell-centre fields (the cell's own on a domain face).  Per
// step the rates are frozen: face f (order -x, +x, -y, +y, -z, +z) of a cell holding n
// ions of a species has the mean lambda_f = n rate_f dt and the faces' counts are
// independent Poisson(lambda_f), drawn per species (M+ then M-) in one of two equivalent
// ways chosen by Lambda = sum lambda_f (summed in face order):
//   Lambda < 10: N ~ Poisson(Lambda) movers, capped at n, from the stream (cell, step,
//     ION, sub = species); each mover then takes the first face whose running sum of
//     lambda exceeds u Lambda, u the stream's next uniform;
//   otherwise: each face's Poisson(lambda_f) from its own stream (cell, step, ION,
//     sub = 2 + 6 species + face), capped at the ions not yet moved.
// Ions crossing a domain face leave and are tallied.  The field is the step's E^{k+1}
// (the prescribed one in the uniform mode).
//
// Three passes: clear the next counts, move (one lane per cell; integer atomics, so the
// result does not depend on their order), copy back.  Each returns at entry once the
// device-side stop rule has halted the run.
#include "device.hpp"
#include "itk.hpp"
#include "poisson.hpp"

namespace itk {
namespace {

template <typename T>
__device__ __forceinline__ void cell_field(const T* E4, const double Eu[3], uint32_t c, double out[3]) {
  if (E4 == nullptr) {
    out[0] = Eu[0];
    out[1] = Eu[1];
    out[2] = Eu[2];
  } else {
    const T* e = E4 + 4 * (size_t)c;
    out[0] = (double)e[0];
    out[1] = (double)e[1];
    out[2] = (double)e[2];
  }
}

__global__ void k_ion_clear(uint32_t* a, uint32_t* b, uint32_t n, Counters* ctr) {
  if (ctr->halt) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) ctr->n_ionbig = 0u;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    a[c] = 0u;
    b[c] = 0u;
  }
}

struct IonMove {
  double Eu[3];
  double mu_ion, D_ion;
};

// Face means lambda_f = n rate_f dt of one species in cell c (face order -x, +x, -y, +y,
// -z, +z), the neighbour of each face and whether it lies inside the grid; returns
// their sum in face order.
template <typename T>
__device__ __forceinline__ double ion_lambdas(const StepConst& K, const T* E4, const IonMove& m, uint32_t c,
                                              int sp, uint32_t cnt, double lam[6], uint32_t nb[6],
                                              bool inside[6]) {
  int ci[3];
  cell_ijk(c, K, ci[0], ci[1], ci[2]);
  const int lim[3] = {K.nx, K.ny, K.nz};
  double Ec[3];
  cell_field<T>(E4, m.Eu, c, Ec);
  const double inv_dx = 1.0 / K.dx;
  const double dr = m.D_ion / (K.dx * K.dx);
  const double q = sp == 0 ? 1.0 : -1.0;
  double L = 0.0;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int a = f >> 1, d = (f & 1) ? 1 : -1;
    int nb3[3] = {ci[0], ci[1], ci[2]};
    nb3[a] += d;
    inside[f] = nb3[a] >= 0 && nb3[a] < lim[a];
    nb[f] = 0u;
    double Ef = Ec[a];
    if (inside[f]) {
      nb[f] = (uint32_t)nb3[0] + (uint32_t)K.nx * ((uint32_t)nb3[1] + (uint32_t)K.ny * (uint32_t)nb3[2]);
      double En[3];
      cell_field<T>(E4, m.Eu, nb[f], En);
      Ef = 0.5 * (Ec[a] + En[a]);
    }
    const double dir = (f & 1) ? 1.0 : -1.0;
    const double v = q * m.mu_ion * Ef;
    const double rate = fmax(0.0, dir * v) * inv_dx + dr;
    lam[f] = (double)cnt * rate * K.dt;
    L += lam[f];
  }
  return L;
}

// Hand one species' face counts to the next counts (or the outflow tally).
__device__ __forceinline__ void ion_apply(const uint32_t kf[6], const uint32_t nb[6], const bool inside[6],
                                          uint32_t c, uint32_t cnt, uint32_t* nxt, uint64_t& out) {
  uint32_t moved = 0u;
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    moved += kf[f];
    if (kf[f] == 0u) continue;
    if (inside[f]) atomicAdd(&nxt[nb[f]], kf[f]);
    else out += (uint64_t)kf[f];
  }
  if (cnt - moved) atomicAdd(&nxt[c], cnt - moved);
}

// Small total means: the Poisson total split over the faces, one lane per cell.  A
// species whose total mean is 10 or more is appended to a list for k_ion_big, which
// holds the large-mean sampler (and its registers) apart.
template <typename T>
__global__ void __launch_bounds__(256) k_ion_move(StepConst K, const T* E4, IonMove m, const uint32_t* np,
                                                 const uint32_t* nm, uint32_t* next_p, uint32_t* next_m,
                                                 uint32_t* big, Counters* ctr) {
  if (ctr->halt) return;
  const uint32_t n = K.ncell;
  uint64_t out[2] = {0, 0};
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const uint32_t n0[2] = {np[c], nm[c]};
    if ((n0[0] | n0[1]) == 0u) continue;
#pragma unroll 1
    for (int sp = 0; sp < 2; ++sp) {
      const uint32_t cnt = n0[sp];
      if (cnt == 0u) continue;
      double lam[6];
      uint32_t nb[6];
      bool inside[6];
      const double L = ion_lambdas<T>(K, E4, m, c, sp, cnt, lam, nb, inside);
      if (!(L > 0.0)) continue;
      if (!(L < 10.0)) {
        big[atomicAdd(&ctr->n_ionbig, 1u)] = (c << 1) | (uint32_t)sp;
        continue;
      }
      uint32_t kf[6] = {0u, 0u, 0u, 0u, 0u, 0u};
      CellStream st;
      st.init(c, K.step, TAG_ION, (uint32_t)sp, K.key);
      int64_t N = poisson_small(L, st);
      if (N > (int64_t)cnt) N = (int64_t)cnt;
      for (int64_t r = 0; r < N; ++r) {
        const double t = u_co(st.next()) * L;
        // the first face whose running sum of lambda exceeds t (static indexing)
        int f = 0;
        double acc = lam[0];
#pragma unroll
        for (int g = 1; g < 6; ++g) {
          if (f == g - 1 && t >= acc) {
            f = g;
            acc += lam[g];
          }
        }
#pragma unroll
        for (int g = 0; g < 6; ++g) kf[g] += f == g ? 1u : 0u;
      }
      ion_apply(kf, nb, inside, c, cnt, sp == 0 ? next_p : next_m, out[sp]);
    }
  }
  const uint64_t op = wave_sum64(out[0]), om = wave_sum64(out[1]);
  if (lane_id() == 0) {
    if (op) atomicAdd(&ctr->ion_out[0], (unsigned long long)op);
    if (om) atomicAdd(&ctr->ion_out[1], (unsigned long long)om);
  }
}

// Large total means: each face's Poisson count from its own stream, capped at the ions
// not yet moved.
template <typename T>
__global__ void __launch_bounds__(256) k_ion_big(StepConst K, const T* E4, IonMove m, const uint32_t* np,
                                                const uint32_t* nm, uint32_t* next_p, uint32_t* next_m,
                                                const uint32_t* big, Counters* ctr) {
  if (ctr->halt) return;
  const uint32_t nbig = ctr->n_ionbig;
  uint64_t out[2] = {0, 0};
  for (uint32_t w = blockIdx.x * blockDim.x + threadIdx.x; w < nbig; w += gridDim.x * blockDim.x) {
    const uint32_t c = big[w] >> 1;
    const int sp = (int)(big[w] & 1u);
    const uint32_t cnt = sp == 0 ? np[c] : nm[c];
    double lam[6];
    uint32_t nb[6];
    bool inside[6];
    (void)ion_lambdas<T>(K, E4, m, c, sp, cnt, lam, nb, inside);
    uint32_t kf[6];
    uint32_t left = cnt;
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      CellStream st;
      st.init(c, K.step, TAG_ION, (uint32_t)(2 + 6 * sp + f), K.key);
      int64_t k = poisson_draw(lam[f], st);
      if (k > (int64_t)left) k = (int64_t)left;
      left -= (uint32_t)k;
      kf[f] = (uint32_t)k;
    }
    ion_apply(kf, nb, inside, c, cnt, sp == 0 ? next_p : next_m, out[sp]);
  }
  const uint64_t op = wave_sum64(out[0]), om = wave_sum64(out[1]);
  if (lane_id() == 0) {
    if (op) atomicAdd(&ctr->ion_out[0], (unsigned long long)op);
    if (om) atomicAdd(&ctr->ion_out[1], (unsigned long long)om);
  }
}

__global__ void k_ion_commit(uint32_t* np, uint32_t* nm, const uint32_t* a, const uint32_t* b, uint32_t n,
                             const Counters* ctr) {
  if (ctr->halt) return;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    np[c] = a[c];
    nm[c] = b[c];
  }
}

int grid_for(uint32_t n, int cap) {
  const uint64_t g = ((uint64_t)n + 255) / 256;
  return (int)(g < 1 ? 1 : (g > (uint64_t)cap ? (uint64_t)cap : g));
}

}  // namespace

hipError_t launch_ion_move(itokmc_ctx* ctx, const StepConst& K, const void* E4) {
  const uint32_t n = ctx->ncell;
  hipStream_t s = ctx->s;
  phase_begin(ctx, PH_IONS);
  k_ion_clear<<<grid_for(n, 4096), 256, 0, s>>>(ctx->ion_next[0], ctx->ion_next[1], n, ctx->ctr);
  IonMove m;
  for (int a = 0; a < 3; ++a) m.Eu[a] = ctx->d.E_uniform[a];
  m.mu_ion = ctx->c.mu_ion;
  m.D_ion = ctx->c.D_ion;
  if (ctx->d.precision == ITOKMC_FP64) {
    k_ion_move<double><<<grid_for(n, 8192), 256, 0, s>>>(K, (const double*)E4, m, ctx->nplus, ctx->nminus,
                                                         ctx->ion_next[0], ctx->ion_next[1], ctx->ion_big,
                                                         ctx->ctr);
    k_ion_big<double><<<1024, 256, 0, s>>>(K, (const double*)E4, m, ctx->nplus, ctx->nminus, ctx->ion_next[0],
                                           ctx->ion_next[1], ctx->ion_big, ctx->ctr);
  } else {
    k_ion_move<float><<<grid_for(n, 8192), 256, 0, s>>>(K, (const float*)E4, m, ctx->nplus, ctx->nminus,
                                                        ctx->ion_next[0], ctx->ion_next[1], ctx->ion_big,
                                                        ctx->ctr);
    k_ion_big<float><<<1024, 256, 0, s>>>(K, (const float*)E4, m, ctx->nplus, ctx->nminus, ctx->ion_next[0],
                                          ctx->ion_next[1], ctx->ion_big, ctx->ctr);
  }
  k_ion_commit<<<grid_for(n, 4096), 256, 0, s>>>(ctx->nplus, ctx->nminus, ctx->ion_next[0], ctx->ion_next[1], n,
                                                 ctx->ctr);
  phase_end(ctx, PH_IONS);
  return hipGetLastError();
}

}  // namespace itk
