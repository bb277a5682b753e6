// Field-coupled (Poisson) mode and CIC transfers.
#include <math.h>

#include "device.hpp"
#include "itk.hpp"

namespace itk {

namespace {

template <typename T>
__device__ __forceinline__ const T* cas(const void* p) { return reinterpret_cast<const T*>(p); }

// Clamped tent weights along one axis about cell centres (i + 1/2): lower node and the
// weight of the upper node; the part of a cloud beyond the outermost centres folds
// into the wall cell.
__device__ __forceinline__ void tent(double xi, int n, int& i0, double& f) {
  double s = xi - 0.5;
  s = s < 0.0 ? 0.0 : s;
  s = s > (double)(n - 1) ? (double)(n - 1) : s;
  if (n == 1) { i0 = 0; f = 0.0; return; }
  int i = (int)floor(s);
  i = i > n - 2 ? n - 2 : i;
  i0 = i;
  f = s - (double)i;
}

template <typename T>
__global__ void k_cic_density(Bank a, const Counters* ctr, int which, StepConst K, double inv_dV,
                              double* out) {
  const uint32_t n = min(ctr->n[which], K.cap);
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t w = a.w[i];
    if (!w) continue;
    const uint32_t c = a.cell[i];
    const double xi[3] = {(double)(c % (uint32_t)K.nx) + (double)cas<T>(a.ox)[i],
                          (double)((c / (uint32_t)K.nx) % (uint32_t)K.ny) + (double)cas<T>(a.oy)[i],
                          (double)(c / ((uint32_t)K.nx * (uint32_t)K.ny)) + (double)cas<T>(a.oz)[i]};
    int i0, j0, k0;
    double fx, fy, fz;
    tent(xi[0], K.nx, i0, fx);
    tent(xi[1], K.ny, j0, fy);
    tent(xi[2], K.nz, k0, fz);
    const double q = (double)w * inv_dV;
    for (int cc = 0; cc < 8; ++cc) {
      const int di = cc & 1, dj = (cc >> 1) & 1, dk = (cc >> 2) & 1;
      const double wt = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
      if (wt == 0.0) continue;
      const int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
      if (ii >= K.nx || jj >= K.ny || kk >= K.nz) continue;
      atomicAdd(&out[(size_t)ii + (size_t)K.nx * ((size_t)jj + (size_t)K.ny * kk)], q * wt);
    }
  }
}

}  // namespace

hipError_t launch_cic_density(itokmc_ctx* ctx, double* out) {
  hipError_t e = hipMemsetAsync(out, 0, sizeof(double) * ctx->ncell, ctx->s);
  if (e != hipSuccess) return e;
  StepConst K = make_const(ctx, 0.0);
  const double inv_dV = 1.0 / (ctx->d.dx * ctx->d.dx * ctx->d.dx);
  if (ctx->d.precision == ITOKMC_FP64)
    k_cic_density<double><<<2048, 256, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, inv_dV, out);
  else
    k_cic_density<float><<<2048, 256, 0, ctx->s>>>(ctx->bank[ctx->cur], ctx->ctr, ctx->cur, K, inv_dV, out);
  return hipGetLastError();
}

size_t field_bytes(const itokmc_grid_desc* d) {
  if (d->field_mode != ITOKMC_FIELD_POISSON) return 0;
  return 256;
}

int field_init(itokmc_ctx* ctx, char*) {
  return set_error(ctx, ITOKMC_EINVAL, "Poisson field mode is not available in this build");
}
int field_transport(itokmc_ctx* ctx, const StepConst&) {
  return set_error(ctx, ITOKMC_EINVAL, "Poisson field mode is not available in this build");
}
const double* field_cell_rates(itokmc_ctx*) { return nullptr; }
int field_get_phi(itokmc_ctx* ctx, double*) { return set_error(ctx, ITOKMC_EINVAL, "no field"); }
int field_set_phi(itokmc_ctx* ctx, const double*) { return set_error(ctx, ITOKMC_EINVAL, "no field"); }
int field_deposit(itokmc_ctx* ctx, int, void*) { return set_error(ctx, ITOKMC_EINVAL, "no field"); }

}  // namespace itk
