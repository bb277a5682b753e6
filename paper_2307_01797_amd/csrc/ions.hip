// Mobile ions on the grid.  The paper moves ions as Ito particles (positive ions along
// E, eq. Vk1 with sgn(Z) = +1) and proposes heavy species as a continuum in its
// future-work section.  Here the ions stay the per-cell integer counts of the reaction
// network and move as a lattice jump process, the first-order upwind finite-volume
// form of the drift-diffusion equation realised with integer jumps: an ion of sign q
// crosses the face towards its neighbour along axis a in direction d (-1, +1) at the rate
//     max(0, d q mu_ion E_face,a) / dx + D_ion / dx^2,
// E_face the mean of the two cell-centre fields (the cell's own on a domain face).  Per
// step the rates are frozen; each face's count is Poisson(n rate dt) with n the cell's
// count before the move, drawn for M+ then M- in the face order -x, +x, -y, +y, -z, +z,
// each from its own stream (cell, step, ION, sub = 6 species + face: a face whose rate
// is a rounding error away from zero shifts no other face's draws), each capped at the
// ions not yet moved.  Ions crossing a domain face leave and are tallied.  The field is
// the step's E^{k+1} (the prescribed one in the uniform mode).
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

__global__ void k_ion_clear(uint32_t* a, uint32_t* b, uint32_t n, const Counters* ctr) {
  if (ctr->halt) return;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    a[c] = 0u;
    b[c] = 0u;
  }
}

struct IonMove {
  double Eu[3];
  double mu_ion, D_ion;
};

template <typename T>
__global__ void __launch_bounds__(256) k_ion_move(StepConst K, const T* E4, IonMove m, const uint32_t* np,
                                                 const uint32_t* nm, uint32_t* next_p, uint32_t* next_m,
                                                 Counters* ctr) {
  if (ctr->halt) return;
  const uint32_t n = K.ncell;
  const double inv_dx = 1.0 / K.dx;
  const double dr = m.D_ion / (K.dx * K.dx);
  const int lim[3] = {K.nx, K.ny, K.nz};
  uint64_t out_p = 0, out_m = 0;
  for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < n; c += gridDim.x * blockDim.x) {
    const uint32_t n0[2] = {np[c], nm[c]};
    if ((n0[0] | n0[1]) == 0u) continue;
    int ci[3];
    cell_ijk(c, K, ci[0], ci[1], ci[2]);
    double Ec[3];
    cell_field<T>(E4, m.Eu, c, Ec);
    for (int sp = 0; sp < 2; ++sp) {
      const double q = sp == 0 ? 1.0 : -1.0;
      uint32_t* nxt = sp == 0 ? next_p : next_m;
      uint32_t left = n0[sp];
      for (int f = 0; f < 6; ++f) {
        const int a = f >> 1, dir = (f & 1) ? 1 : -1;
        int nb3[3] = {ci[0], ci[1], ci[2]};
        nb3[a] += dir;
        const bool inside = nb3[a] >= 0 && nb3[a] < lim[a];
        double Ef = Ec[a];
        uint32_t nb = 0u;
        if (inside) {
          nb = (uint32_t)nb3[0] + (uint32_t)K.nx * ((uint32_t)nb3[1] + (uint32_t)K.ny * (uint32_t)nb3[2]);
          double En[3];
          cell_field<T>(E4, m.Eu, nb, En);
          Ef = 0.5 * (Ec[a] + En[a]);
        }
        const double v = q * m.mu_ion * Ef;
        const double rate = fmax(0.0, (double)dir * v) * inv_dx + dr;
        CellStream st;
        st.init(c, K.step, TAG_ION, (uint32_t)(6 * sp + f), K.key);
        int64_t kf = poisson_draw((double)n0[sp] * rate * K.dt, st);
        if (kf > (int64_t)left) kf = (int64_t)left;
        left -= (uint32_t)kf;
        if (kf == 0) continue;
        if (inside) atomicAdd(&nxt[nb], (uint32_t)kf);
        else if (sp == 0) out_p += (uint64_t)kf;
        else out_m += (uint64_t)kf;
      }
      if (left) atomicAdd(&nxt[c], left);
    }
  }
  out_p = wave_sum64(out_p);
  out_m = wave_sum64(out_m);
  if (lane_id() == 0) {
    if (out_p) atomicAdd(&ctr->ion_out[0], (unsigned long long)out_p);
    if (out_m) atomicAdd(&ctr->ion_out[1], (unsigned long long)out_m);
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
  if (ctx->d.precision == ITOKMC_FP64)
    k_ion_move<double><<<grid_for(n, 8192), 256, 0, s>>>(K, (const double*)E4, m, ctx->nplus, ctx->nminus,
                                                         ctx->ion_next[0], ctx->ion_next[1], ctx->ctr);
  else
    k_ion_move<float><<<grid_for(n, 8192), 256, 0, s>>>(K, (const float*)E4, m, ctx->nplus, ctx->nminus,
                                                        ctx->ion_next[0], ctx->ion_next[1], ctx->ctr);
  k_ion_commit<<<grid_for(n, 4096), 256, 0, s>>>(ctx->nplus, ctx->nminus, ctx->ion_next[0], ctx->ion_next[1], n,
                                                 ctx->ctr);
  phase_end(ctx, PH_IONS);
  return hipGetLastError();
}

}  // namespace itk
