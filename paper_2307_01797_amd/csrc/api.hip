// C ABI of the itokmc library: context and arena layout, step orchestration,
// diagnostics and state exchange.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <cmath>
#include <vector>

#include "device.hpp"
#include "itk.hpp"

namespace itk {

int set_error(itokmc_ctx* ctx, int code, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->err = buf;
  }
  return code;
}

int check_hip(itokmc_ctx* ctx, hipError_t e, const char* what) {
  if (e == hipSuccess) return ITOKMC_OK;
  return set_error(ctx, ITOKMC_EHIP, "%s: %s", what, hipGetErrorString(e));
}

static double mobility(const itokmc_coeffs& c, double E) {
  const double Ec = E > c.E_floor ? E : c.E_floor;
  return c.mu_a * pow(Ec / c.mu_E0, c.mu_b);
}

void phase_begin(itokmc_ctx* ctx, int phase) {
  if (!ctx->profiling) return;
  hipEvent_t b, e;
  if (ctx->ev_free.size() >= 2) {
    b = ctx->ev_free.back(); ctx->ev_free.pop_back();
    e = ctx->ev_free.back(); ctx->ev_free.pop_back();
  } else {
    hipEventCreate(&b);
    hipEventCreate(&e);
  }
  hipEventRecord(b, ctx->s);
  ctx->ev_used.push_back({phase, {b, e}});
}

void phase_end(itokmc_ctx* ctx, int phase) {
  if (!ctx->profiling || ctx->ev_used.empty()) return;
  auto& last = ctx->ev_used.back();
  if (last.first != phase) return;
  hipEventRecord(last.second.second, ctx->s);
}

static void phase_collect(itokmc_ctx* ctx) {
  if (ctx->ev_used.empty()) return;
  hipStreamSynchronize(ctx->s);
  for (auto& u : ctx->ev_used) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, u.second.first, u.second.second) == hipSuccess) {
      ctx->phase_ms[u.first] += ms;
      ctx->phase_calls[u.first] += 1;
    }
    ctx->ev_free.push_back(u.second.first);
    ctx->ev_free.push_back(u.second.second);
  }
  ctx->ev_used.clear();
}

// Electron-ion and ion-ion recombination rates in a cell of edge dx at field magnitude
// Em: k_ep = beta_ep T_e^beta_ep_b / dV with T_e = max(300 K, Te_a (max(Em,
// E_floor)/mu_E0)^Te_b), k_np = beta_np / dV (0 when the coefficient is 0).
void recomb_rates(const itokmc_coeffs& c, double Em, double dx, double k[2]) {
  const double dV = dx * dx * dx;
  k[0] = 0.0;
  if (c.beta_ep > 0.0) {
    const double E = Em > c.E_floor ? Em : c.E_floor;
    const double Te = fmax(300.0, c.Te_a * pow(E / c.mu_E0, c.Te_b));
    k[0] = c.beta_ep * pow(Te, c.beta_ep_b) / dV;
  }
  k[1] = c.beta_np > 0.0 ? c.beta_np / dV : 0.0;
}

void uniform_consts(const itokmc_grid_desc& d, const itokmc_coeffs& c, double dt,
                    double drift[3], double* diff, double k[5]) {
  *diff = sqrt(2.0 * c.D * dt) / d.dx;
  const double* E = d.E_uniform;
  const double Em = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
  const double mu = mobility(c, Em);
  for (int a = 0; a < 3; ++a) drift[a] = (-mu * E[a] * dt) / d.dx;
  const double alpha = Em > 0.0 ? c.alpha_A * exp(-c.alpha_B / Em) : 0.0;
  const double v = mu * Em;
  k[0] = alpha * v;
  k[1] = c.eta * v;
  k[2] = c.kgamma_ratio * k[0];
  recomb_rates(c, Em, d.dx, k + 3);
}

StepConst make_const(const itokmc_ctx* ctx, double dt) {
  StepConst k{};
  k.nx = ctx->d.nx; k.ny = ctx->d.ny; k.nz = ctx->d.nz;
  div_magic((uint32_t)k.nx, &k.mdx, &k.sdx);
  div_magic((uint32_t)k.ny, &k.mdy, &k.sdy);
  k.ncell = ctx->ncell;
  k.cap = (uint32_t)ctx->cap;
  k.step = ctx->step;
  k.key = Key{ctx->d.seed, ctx->d.realization};
  k.dx = ctx->d.dx;
  k.dt = dt;
  if (ctx->have_coeffs) {
    if (ctx->d.field_mode == ITOKMC_FIELD_UNIFORM) {
      uniform_consts(ctx->d, ctx->c, dt, k.drift, &k.diff, k.k);
    } else {
      k.diff = sqrt(2.0 * ctx->c.D * dt) / ctx->d.dx;
    }
  }
  return k;
}

// ---- arena layout ------------------------------------------------------------------

struct Layout {
  size_t off[40];
  size_t total;
};

static size_t al(size_t x) { return (x + 255) & ~(size_t)255; }

bool valid_desc(const itokmc_grid_desc* d) {
  if (!d) return false;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return false;
  const uint64_t nc = (uint64_t)d->nx * d->ny * d->nz;
  if (nc > (1ull << 24)) return false;
  if (!(d->dx > 0.0)) return false;
  if (d->precision != ITOKMC_FP32 && d->precision != ITOKMC_FP64) return false;
  if (d->field_mode != ITOKMC_FIELD_UNIFORM && d->field_mode != ITOKMC_FIELD_POISSON) return false;
  if (d->kmc_mode != ITOKMC_KMC_HYBRID && d->kmc_mode != ITOKMC_KMC_PURE_TAU) return false;
  if (d->shape != ITOKMC_SHAPE_CIC && d->shape != ITOKMC_SHAPE_TSC) return false;
  if (d->n_new < 1 || d->n_new > 64) return false;
  if (d->n_ppc < 0 || d->n_ppc > 64) return false;
  if (d->kmc_nc < 0 || d->kmc_nssa < 1) return false;
  if (!(d->kmc_eps > 0.0)) return false;
  if (d->max_particles < 1 || d->max_particles > 0x7FFFFFFFull) return false;
  return true;
}

// index: 0..1 banks handled separately; per-bank arrays follow
static void layout(const itokmc_grid_desc* d, Layout* L) {
  const uint64_t nc = (uint64_t)d->nx * d->ny * d->nz;
  const uint64_t cap = d->max_particles;
  const size_t T = d->precision == ITOKMC_FP64 ? 8 : 4;
  size_t o = 0;
  int i = 0;
  auto put = [&](size_t bytes) { L->off[i++] = o; o += al(bytes); };
  for (int b = 0; b < 2; ++b) {
    put(cap * 4);      // cell
    put(cap * T);      // ox
    put(cap * T);      // oy
    put(cap * T);      // oz
    put(cap * 4);      // w
    put(cap * 8);      // id
    put(cap * 4);      // rank
  }
  put(nc * 8);         // 14 cellacc
  put((nc + 1) * 4);   // 15 start
  put(nc * 4);         // 16 occ
  put(nc * 12);        // 17 occ_fires
  put(nc * 4);         // 18 nplus
  put(nc * 4);         // 19 nminus
  put(nc * 4);         // 20 ngamma
  put(nc * 4);         // 21 dN
  put(nc * 4);         // 22 work
  put(scan_scratch_words(nc) * 4);    // 23 scan scratch
  put(sizeof(Counters));              // 24 counters
  put(64);                            // 25 reduction scratch
  put(field_bytes(d));                // 26 field data
  put(nc * 4);                        // 27 cbase
  put(nc * 4);                        // 28 big
  put((nc / 2048 + 2) * 4);           // 29 scan tile flags
  put(nc * 4);                        // 30 cells for the full KMC pass
  put(d->field_mode == ITOKMC_FIELD_POISSON ? nc * 24 : 64);  // 31 rates for the full pass
  put(nc * 4);                        // 32 huge (large merge list)
  put(nc * 4);                        // 33 cells for the wavefront coupling pass
  put(nc * 4);                        // 34 cells to merge after the light pass
  put(d->field_mode == ITOKMC_FIELD_POISSON ? cap * T : 64);  // 35 mobility per particle
  put(nc * 4);                        // 36 positive ions after a transport move
  put(nc * 4);                        // 37 negative ions after a transport move
  put(nc * 8);                        // 38 ion species of large total mean (two per cell)
  L->total = o;
}

int check_coeffs(const itokmc_coeffs* c, std::string* why) {
  const double v[] = {c->mu_a, c->mu_E0, c->mu_b, c->E_floor, c->D, c->alpha_A, c->alpha_B,
                      c->eta, c->kgamma_ratio, c->photon_l1, c->photon_l2, c->beta_ep,
                      c->beta_ep_b, c->Te_a, c->Te_b, c->beta_np, c->mu_ion, c->D_ion};
  for (double x : v)
    if (!isfinite(x)) { *why = "non-finite coefficient"; return ITOKMC_EINVAL; }
  if (c->mu_a < 0 || !(c->mu_E0 > 0) || !(c->E_floor > 0) || c->D < 0 || c->alpha_A < 0 ||
      c->eta < 0 || c->kgamma_ratio < 0 || c->beta_ep < 0 || c->Te_a < 0 || c->beta_np < 0 ||
      c->mu_ion < 0 || c->D_ion < 0) {
    *why = "negative transport or rate coefficient";
    return ITOKMC_EINVAL;
  }
  if (c->kgamma_ratio > 0 && !(c->photon_l1 > 0 && c->photon_l2 >= c->photon_l1)) {
    *why = "invalid photon absorption lengths";
    return ITOKMC_EINVAL;
  }
  return ITOKMC_OK;
}

}  // namespace itk

using namespace itk;

extern "C" {

size_t itokmc_arena_bytes(const itokmc_grid_desc* desc) {
  if (!valid_desc(desc)) return 0;
  Layout L;
  layout(desc, &L);
  return L.total;
}

int itokmc_init_grid(itokmc_ctx** out, const itokmc_grid_desc* desc, void* arena,
                     size_t arena_bytes, void* stream) {
  if (!out) return ITOKMC_EINVAL;
  *out = nullptr;
  if (!valid_desc(desc)) return ITOKMC_EINVAL;
  Layout L;
  layout(desc, &L);
  if (!arena || ((uintptr_t)arena & 255)) return ITOKMC_EINVAL;
  if (arena_bytes < L.total) return ITOKMC_ENOMEM;
  itokmc_ctx* ctx = new itokmc_ctx();
  ctx->d = *desc;
  ctx->s = (hipStream_t)stream;
  ctx->arena = (char*)arena;
  ctx->arena_bytes = arena_bytes;
  ctx->ncell = (uint32_t)((uint64_t)desc->nx * desc->ny * desc->nz);
  ctx->cap = desc->max_particles;
  char* a = ctx->arena;
  for (int b = 0; b < 2; ++b) {
    Bank& k = ctx->bank[b];
    const int o = 7 * b;
    k.cell = (uint32_t*)(a + L.off[o]);
    k.ox = a + L.off[o + 1];
    k.oy = a + L.off[o + 2];
    k.oz = a + L.off[o + 3];
    k.w = (uint32_t*)(a + L.off[o + 4]);
    k.id = (uint64_t*)(a + L.off[o + 5]);
    k.rank = (uint32_t*)(a + L.off[o + 6]);
  }
  ctx->cellacc = (unsigned long long*)(a + L.off[14]);
  ctx->start = (uint32_t*)(a + L.off[15]);
  ctx->occ = (uint32_t*)(a + L.off[16]);
  ctx->occ_fires = (uint32_t*)(a + L.off[17]);
  ctx->nplus = (uint32_t*)(a + L.off[18]);
  ctx->nminus = (uint32_t*)(a + L.off[19]);
  ctx->ngamma = (uint32_t*)(a + L.off[20]);
  ctx->dN = (int32_t*)(a + L.off[21]);
  ctx->work = (uint32_t*)(a + L.off[22]);
  ctx->blocksums = (uint32_t*)(a + L.off[23]);
  ctx->ctr = (Counters*)(a + L.off[24]);
  ctx->reduce = (unsigned long long*)(a + L.off[25]);
  ctx->field = a + L.off[26];
  ctx->cbase = (uint32_t*)(a + L.off[27]);
  ctx->big = (uint32_t*)(a + L.off[28]);
  ctx->tiles = (uint32_t*)(a + L.off[29]);
  ctx->heavy = (uint32_t*)(a + L.off[30]);
  ctx->rates = (double*)(a + L.off[31]);
  ctx->huge = (uint32_t*)(a + L.off[32]);
  ctx->cfull = (uint32_t*)(a + L.off[33]);
  ctx->cmerge = (uint32_t*)(a + L.off[34]);
  ctx->mu_p = a + L.off[35];
  ctx->ion_next[0] = (uint32_t*)(a + L.off[36]);
  ctx->ion_next[1] = (uint32_t*)(a + L.off[37]);
  ctx->ion_big = (uint32_t*)(a + L.off[38]);
  const size_t nb = ctx->ncell;
  hipError_t e = hipSuccess;
  if (e == hipSuccess) e = hipMemsetAsync(ctx->cellacc, 0, nb * 8, ctx->s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->nplus, 0, nb * 4, ctx->s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->nminus, 0, nb * 4, ctx->s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->ngamma, 0, nb * 4, ctx->s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->ctr, 0, sizeof(Counters), ctx->s);
  if (e == hipSuccess) e = hipMemsetAsync(ctx->tiles, 0, (nb / 2048 + 2) * 4, ctx->s);
  if (e == hipSuccess) e = hipHostMalloc((void**)&ctx->host_ctr, sizeof(Counters), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete ctx;
    return ITOKMC_EHIP;
  }
  if (desc->field_mode == ITOKMC_FIELD_POISSON) {
    const int rc = field_init(ctx, (char*)ctx->field);
    if (rc != ITOKMC_OK) {
      (void)hipHostFree(ctx->host_ctr);
      delete ctx;
      return rc;
    }
  }
  *out = ctx;
  return ITOKMC_OK;
}

int itokmc_set_coefficients(itokmc_ctx* ctx, const itokmc_coeffs* c) {
  if (!ctx || !c) return ITOKMC_EINVAL;
  std::string why;
  if (check_coeffs(c, &why)) return set_error(ctx, ITOKMC_EINVAL, "%s", why.c_str());
  ctx->c = *c;
  ctx->have_coeffs = true;
  return ITOKMC_OK;
}

int itokmc_check_coefficients(const itokmc_coeffs* c) {
  if (!c) return ITOKMC_EINVAL;
  std::string why;
  return check_coeffs(c, &why);
}

static int mark_unbinned(itokmc_ctx* ctx) {
  // the bin accumulator must be all zero between steps; recount before reacting
  return check_hip(ctx, hipMemsetAsync(ctx->cellacc, 0, (size_t)ctx->ncell * 8, ctx->s), "memset");
}

int itokmc_seed_particles(itokmc_ctx* ctx, const itokmc_seed_desc* sd) {
  if (!ctx || !sd) return ITOKMC_EINVAL;
  if (!(sd->sigma > 0.0)) return set_error(ctx, ITOKMC_EINVAL, "sigma must be positive");
  hipError_t e;
  if (sd->kind == ITOKMC_SEED_GAUSSIAN) e = launch_seed_gaussian(ctx, sd);
  else if (sd->kind == ITOKMC_SEED_NEUTRAL) e = launch_seed_neutral(ctx, sd);
  else return set_error(ctx, ITOKMC_EINVAL, "unknown seed kind");
  int rc = check_hip(ctx, e, "seed");
  if (rc) return rc;
  ctx->field_valid = false;
  return mark_unbinned(ctx);
}

// ---- step orchestration --------------------------------------------------------------

int itokmc_transport(itokmc_ctx* ctx, double dt) {
  if (!ctx) return ITOKMC_EINVAL;
  if (!ctx->have_coeffs) return set_error(ctx, ITOKMC_EINVAL, "coefficients not set");
  if (!(dt > 0.0)) return set_error(ctx, ITOKMC_EINVAL, "dt must be positive");
  StepConst k = make_const(ctx, dt);
  int rc;
  if (ctx->d.field_mode == ITOKMC_FIELD_UNIFORM) {
    if (ctx->binned) {
      // transport twice without react: re-zero the bins first
      rc = mark_unbinned(ctx);
      if (rc) return rc;
    }
    phase_begin(ctx, PH_PUSH);
    rc = check_hip(ctx, launch_push_uniform(ctx, k), "push");
    phase_end(ctx, PH_PUSH);
    if (!rc && mobile_ions(ctx)) rc = check_hip(ctx, launch_ion_move(ctx, k, nullptr), "ions");
  } else {
    if (ctx->binned) {
      rc = mark_unbinned(ctx);
      if (rc) return rc;
    }
    rc = field_transport(ctx, k);
  }
  if (rc) return rc;
  ctx->binned = true;
  return ITOKMC_OK;
}

int itokmc_react(itokmc_ctx* ctx, double dt) {
  if (!ctx) return ITOKMC_EINVAL;
  if (!ctx->have_coeffs) return set_error(ctx, ITOKMC_EINVAL, "coefficients not set");
  if (!(dt > 0.0)) return set_error(ctx, ITOKMC_EINVAL, "dt must be positive");
  StepConst k = make_const(ctx, dt);
  int rc;
  if (!ctx->binned) {
    phase_begin(ctx, PH_COUNT);
    rc = check_hip(ctx, launch_count(ctx), "count");
    phase_end(ctx, PH_COUNT);
    if (rc) return rc;
  }
  phase_begin(ctx, PH_PHOTON);
  rc = check_hip(ctx, launch_photons(ctx, k), "photons");
  phase_end(ctx, PH_PHOTON);
  phase_begin(ctx, PH_SCAN);
  if (!rc) rc = check_hip(ctx, launch_scan(ctx), "scan");
  phase_end(ctx, PH_SCAN);
  phase_begin(ctx, PH_SCATTER);
  if (!rc) rc = check_hip(ctx, launch_scatter(ctx), "scatter");
  phase_end(ctx, PH_SCATTER);
  FieldRates fr{};
  if (ctx->d.field_mode == ITOKMC_FIELD_POISSON) fr = field_rates(ctx);
  phase_begin(ctx, PH_KMC);
  if (!rc) rc = check_hip(ctx, launch_kmc_step(ctx, k, fr), "kmc");
  phase_end(ctx, PH_KMC);
  phase_begin(ctx, PH_COUPLE_LIGHT);  // ended inside: light pass, wavefront pass, merge tiers
  if (!rc) rc = check_hip(ctx, launch_couple(ctx, k), "couple");
  if (rc) return rc;
  ctx->cur = 1 - ctx->cur;
  ctx->step += 1;
  ctx->binned = false;
  return ITOKMC_OK;
}

int itokmc_step(itokmc_ctx* ctx, uint32_t nsteps, double dt) {
  if (!ctx) return ITOKMC_EINVAL;
  for (uint32_t i = 0; i < nsteps; ++i) {
    int rc = itokmc_transport(ctx, dt);
    if (rc) return rc;
    rc = itokmc_react(ctx, dt);
    if (rc) return rc;
  }
  return ITOKMC_OK;
}

// Self-consistent form of the stop rule: the field solve already synchronises with the
// host every refinement cycle, so the steps run one at a time and the host reads the
// device's decision (4 bytes) after each; no step is enqueued past the one that stops.
static int step_until_field(itokmc_ctx* ctx, uint32_t nsteps, double dt, uint64_t stop_particles,
                            uint32_t* steps_done) {
  int rc = check_hip(ctx, launch_stop_begin(ctx), "stop rule");
  uint32_t done = 0;
  uint32_t* halt = &ctx->host_ctr->halt;
  while (!rc && done < nsteps) {
    rc = itokmc_transport(ctx, dt);
    if (!rc) rc = itokmc_react(ctx, dt);
    if (!rc) rc = check_hip(ctx, launch_stop_step(ctx, stop_particles), "stop rule");
    if (rc) break;
    ++done;
    hipError_t e = hipMemcpyAsync(halt, &ctx->ctr->halt, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->s);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->s);
    rc = check_hip(ctx, e, "stop rule");
    if (!rc && *halt) break;
  }
  hipError_t e = launch_stop_end(ctx);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->s);
  const int rc2 = check_hip(ctx, e, "stop rule");
  *steps_done = done;
  return rc ? rc : rc2;
}

int itokmc_step_until(itokmc_ctx* ctx, uint32_t nsteps, double dt, uint64_t stop_particles,
                      uint32_t* steps_done) {
  if (!ctx || !steps_done) return ITOKMC_EINVAL;
  if (!ctx->have_coeffs) return set_error(ctx, ITOKMC_EINVAL, "coefficients not set");
  if (!(dt > 0.0)) return set_error(ctx, ITOKMC_EINVAL, "dt must be positive");
  *steps_done = 0;
  if (nsteps == 0) return ITOKMC_OK;
  if (ctx->d.field_mode == ITOKMC_FIELD_POISSON) return step_until_field(ctx, nsteps, dt, stop_particles, steps_done);
  const uint32_t step0 = ctx->step;
  const int cur0 = ctx->cur;
  int rc = check_hip(ctx, launch_stop_begin(ctx), "stop rule");
  // every step is enqueued; once the rule has stopped the run on the device, the
  // kernels of the remaining steps return at entry
  for (uint32_t i = 0; i < nsteps && !rc; ++i) {
    rc = itokmc_transport(ctx, dt);
    if (!rc) rc = itokmc_react(ctx, dt);
    if (!rc) rc = check_hip(ctx, launch_stop_step(ctx, stop_particles), "stop rule");
  }
  uint32_t done = 0;
  hipError_t e = hipMemcpyAsync(&done, &ctx->ctr->steps_done, sizeof(done), hipMemcpyDeviceToHost, ctx->s);
  if (e == hipSuccess) e = launch_stop_end(ctx);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->s);
  const int rc2 = check_hip(ctx, e, "stop rule");
  if (rc) return rc;
  if (rc2) return rc2;
  // the host enqueued nsteps steps; the state is that of the steps taken
  ctx->step = step0 + done;
  ctx->cur = (done & 1u) ? 1 - cur0 : cur0;
  ctx->binned = false;
  *steps_done = done;
  return ITOKMC_OK;
}

int itokmc_stable_dt(itokmc_ctx* ctx, const itokmc_dt_rule* r, double* out) {
  if (!ctx || !r || !out) return ITOKMC_EINVAL;
  if (!ctx->have_coeffs) return set_error(ctx, ITOKMC_EINVAL, "coefficients not set");
  const auto bad = [](double f) { return !(f >= 0.0) || !std::isfinite(f); };
  if (!(r->dt_max > 0.0) || !std::isfinite(r->dt_max) || bad(r->c_drift) || bad(r->c_diff) ||
      bad(r->c_ion))
    return set_error(ctx, ITOKMC_EINVAL, "time-step rule: dt_max > 0 and finite factors >= 0");
  const itokmc_coeffs& c = ctx->c;
  if ((r->c_drift > 0.0 || r->c_ion > 0.0) && c.mu_b < -1.0)
    return set_error(ctx, ITOKMC_EINVAL, "time-step rule: the field bound needs mu_b >= -1");
  double Em = 0.0;
  if (ctx->d.field_mode == ITOKMC_FIELD_UNIFORM) {
    const double* E = ctx->d.E_uniform;
    Em = sqrt(E[0] * E[0] + E[1] * E[1] + E[2] * E[2]);
  } else {
    const int rc = field_max(ctx, &Em);
    if (rc) return rc;
  }
  const double dx = ctx->d.dx;
  const double v = mobility(c, Em) * Em;
  double dt = r->dt_max;
  if (r->c_drift > 0.0 && v > 0.0) dt = fmin(dt, r->c_drift * dx / v);
  if (r->c_diff > 0.0 && c.D > 0.0) dt = fmin(dt, r->c_diff * dx * dx / (2.0 * c.D));
  const double nu = Em > 0.0 ? c.alpha_A * exp(-c.alpha_B / Em) * v : 0.0;
  if (r->c_ion > 0.0 && nu > 0.0) dt = fmin(dt, r->c_ion / nu);
  out[0] = dt;
  out[1] = Em;
  return ITOKMC_OK;
}

int itokmc_step_adaptive(itokmc_ctx* ctx, const itokmc_dt_rule* r, uint32_t nsteps, double* dts) {
  if (!ctx) return ITOKMC_EINVAL;
  for (uint32_t i = 0; i < nsteps; ++i) {
    double q[2];
    int rc = itokmc_stable_dt(ctx, r, q);
    if (rc) return rc;
    if (dts) dts[i] = q[0];
    rc = itokmc_transport(ctx, q[0]);
    if (rc) return rc;
    rc = itokmc_react(ctx, q[0]);
    if (rc) return rc;
  }
  return ITOKMC_OK;
}

int itokmc_set_step(itokmc_ctx* ctx, uint32_t step) {
  if (!ctx) return ITOKMC_EINVAL;
  ctx->step = step;
  return ITOKMC_OK;
}

int itokmc_deposit(itokmc_ctx* ctx, int what, void* dev_out) {
  if (!ctx || !dev_out) return ITOKMC_EINVAL;
  const size_t nb = ctx->ncell;
  hipError_t e = hipSuccess;
  switch (what) {
    case ITOKMC_Q_NGP_WEIGHT: e = launch_ngp(ctx, (uint32_t*)dev_out); break;
    case ITOKMC_Q_NPLUS: e = hipMemcpyAsync(dev_out, ctx->nplus, nb * 4, hipMemcpyDeviceToDevice, ctx->s); break;
    case ITOKMC_Q_NMINUS: e = hipMemcpyAsync(dev_out, ctx->nminus, nb * 4, hipMemcpyDeviceToDevice, ctx->s); break;
    case ITOKMC_Q_NGAMMA: e = hipMemcpyAsync(dev_out, ctx->ngamma, nb * 4, hipMemcpyDeviceToDevice, ctx->s); break;
    case ITOKMC_Q_FIRES: e = launch_fires_dense(ctx, (uint32_t*)dev_out); break;
    case ITOKMC_Q_CIC_DENSITY: e = launch_cic_density(ctx, (double*)dev_out); break;
    case ITOKMC_Q_RHO: e = launch_rho(ctx, (double*)dev_out); break;
    case ITOKMC_Q_PHI: case ITOKMC_Q_EX: case ITOKMC_Q_EY: case ITOKMC_Q_EZ:
      if (ctx->d.field_mode != ITOKMC_FIELD_POISSON)
        return set_error(ctx, ITOKMC_EINVAL, "no field in uniform mode");
      return field_deposit(ctx, what, dev_out);
    default: return set_error(ctx, ITOKMC_EINVAL, "unknown deposit selector %d", what);
  }
  return check_hip(ctx, e, "deposit");
}

int itokmc_diagnostics(itokmc_ctx* ctx, itokmc_diag* out) {
  if (!ctx || !out) return ITOKMC_EINVAL;
  unsigned long long* scratch = ctx->reduce;
  hipError_t e = hipMemsetAsync(scratch, 0, 64, ctx->s);
  if (e == hipSuccess) e = launch_reduce_particles(ctx, scratch);
  if (e == hipSuccess) e = launch_reduce_cells(ctx, scratch + 2);
  unsigned long long host[4] = {0, 0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(host, scratch, 32, hipMemcpyDeviceToHost, ctx->s);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->host_ctr, ctx->ctr, sizeof(Counters), hipMemcpyDeviceToHost, ctx->s);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->s);
  int rc = check_hip(ctx, e, "diagnostics");
  if (rc) return rc;
  const Counters& c = *ctx->host_ctr;
  memset(out, 0, sizeof(*out));
  out->n_particles = host[0];
  out->weight = host[1];
  out->n_plus = (int64_t)host[2];
  out->n_minus = (int64_t)host[3];
  out->charge = (int64_t)host[2] - (int64_t)host[1] - (int64_t)host[3];
  out->outflow_weight = c.outflow;
  for (int r = 0; r < 5; ++r) out->fires[r] = c.fires[r];
  out->photons_emitted = c.ph_emitted;
  out->photons_absorbed = c.ph_absorbed;
  out->photons_lost = c.ph_lost;
  out->created = c.created;
  out->removed_weight = c.removed;
  out->merged_cells = c.merged;
  out->step = ctx->step;
  out->solver_cycles = ctx->last_cycles;
  out->solver_relres = ctx->last_relres;
  out->rho_sum = 1.602176634e-19 * (double)out->charge;
  out->overflow = c.overflow;
  out->particle_steps = c.pushed;
  out->merge_skipped = c.merge_skipped;
  out->occupied_cells = c.n_occ;
  out->queued_cells = c.n_work;
  out->wave_cells = c.n_cfull + c.n_cmerge;
  out->ion_outflow_plus = c.ion_out[0];
  out->ion_outflow_minus = c.ion_out[1];
  out->couple_pieces = c.couple_pieces;
  out->solver_cycles_total = ctx->total_cycles;
  out->solves_total = ctx->total_solves;
  if (c.overflow) return set_error(ctx, ITOKMC_ECAPACITY, "capacity exceeded (flags %u)", c.overflow);
  return ITOKMC_OK;
}

int itokmc_get_particles(itokmc_ctx* ctx, uint64_t* n, uint32_t* cell, double* off, uint32_t* w,
                         uint64_t* id) {
  if (!ctx || !n) return ITOKMC_EINVAL;
  Counters hc;
  hipError_t e = hipMemcpyAsync(&hc, ctx->ctr, sizeof(Counters), hipMemcpyDeviceToHost, ctx->s);
  if (e == hipSuccess) e = hipStreamSynchronize(ctx->s);
  int rc = check_hip(ctx, e, "get_particles");
  if (rc) return rc;
  const uint32_t N = hc.n[ctx->cur] < ctx->cap ? hc.n[ctx->cur] : (uint32_t)ctx->cap;
  const Bank& b = ctx->bank[ctx->cur];
  std::vector<uint32_t> hw(N), hc_(N);
  std::vector<uint64_t> hid(N);
  const bool f64 = ctx->d.precision == ITOKMC_FP64;
  const size_t T = f64 ? 8 : 4;
  std::vector<char> ho[3];
  for (int a = 0; a < 3; ++a) ho[a].resize((size_t)N * T);
  if (N) {
    e = copy_on(ctx->s, hw.data(), b.w, (size_t)N * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = copy_on(ctx->s, hc_.data(), b.cell, (size_t)N * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = copy_on(ctx->s, hid.data(), b.id, (size_t)N * 8, hipMemcpyDeviceToHost);
    void* src[3] = {b.ox, b.oy, b.oz};
    for (int a = 0; a < 3 && e == hipSuccess; ++a)
      e = copy_on(ctx->s, ho[a].data(), src[a], (size_t)N * T, hipMemcpyDeviceToHost);
    rc = check_hip(ctx, e, "get_particles copy");
    if (rc) return rc;
  }
  uint64_t live = 0;
  for (uint32_t i = 0; i < N; ++i) {
    if (hw[i] == 0) continue;
    if (cell || off || w || id) {
      if (cell) cell[live] = hc_[i];
      if (w) w[live] = hw[i];
      if (id) id[live] = hid[i];
      if (off)
        for (int a = 0; a < 3; ++a)
          off[3 * live + a] = f64 ? ((const double*)ho[a].data())[i] : (double)((const float*)ho[a].data())[i];
    }
    ++live;
  }
  *n = live;
  return ITOKMC_OK;
}

int itokmc_set_particles(itokmc_ctx* ctx, uint64_t n, const uint32_t* cell, const double* off,
                         const uint32_t* w, const uint64_t* id) {
  if (!ctx) return ITOKMC_EINVAL;
  if (n > ctx->cap) return set_error(ctx, ITOKMC_ECAPACITY, "too many particles");
  if (n && (!cell || !off || !w || !id)) return ITOKMC_EINVAL;
  for (uint64_t i = 0; i < n; ++i) {
    if (cell[i] >= ctx->ncell || w[i] == 0) return set_error(ctx, ITOKMC_EINVAL, "bad particle %llu", (unsigned long long)i);
    for (int a = 0; a < 3; ++a)
      if (!(off[3 * i + a] >= 0.0 && off[3 * i + a] < 1.0))
        return set_error(ctx, ITOKMC_EINVAL, "offset out of [0,1) at particle %llu", (unsigned long long)i);
  }
  const bool f64 = ctx->d.precision == ITOKMC_FP64;
  const Bank& b = ctx->bank[ctx->cur];
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (n) {
    std::vector<char> ho[3];
    for (int a = 0; a < 3; ++a) {
      ho[a].resize((size_t)n * (f64 ? 8 : 4));
      for (uint64_t i = 0; i < n; ++i) {
        if (f64) ((double*)ho[a].data())[i] = off[3 * i + a];
        else {
          float f = (float)off[3 * i + a];
          ((float*)ho[a].data())[i] = f < 1.0f ? f : 0x1.fffffep-1f;
        }
      }
    }
    void* dst[3] = {b.ox, b.oy, b.oz};
    if (e == hipSuccess) e = copy_on(ctx->s, b.cell, cell, n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = copy_on(ctx->s, b.w, w, n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = copy_on(ctx->s, b.id, id, n * 8, hipMemcpyHostToDevice);
    for (int a = 0; a < 3 && e == hipSuccess; ++a) e = copy_on(ctx->s, dst[a], ho[a].data(), ho[a].size(), hipMemcpyHostToDevice);
  }
  const uint32_t nn = (uint32_t)n;
  if (e == hipSuccess) e = copy_on(ctx->s, &ctx->ctr->n[ctx->cur], &nn, 4, hipMemcpyHostToDevice);
  int rc = check_hip(ctx, e, "set_particles");
  if (rc) return rc;
  ctx->binned = false;
  ctx->field_valid = false;
  return mark_unbinned(ctx);
}

static uint32_t* counts_ptr(itokmc_ctx* ctx, int which) {
  switch (which) {
    case ITOKMC_Q_NPLUS: return ctx->nplus;
    case ITOKMC_Q_NMINUS: return ctx->nminus;
    case ITOKMC_Q_NGAMMA: return ctx->ngamma;
    default: return nullptr;
  }
}

int itokmc_get_counts(itokmc_ctx* ctx, int which, uint32_t* host) {
  if (!ctx || !host) return ITOKMC_EINVAL;
  uint32_t* p = counts_ptr(ctx, which);
  if (!p) return set_error(ctx, ITOKMC_EINVAL, "bad count selector");
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (e == hipSuccess) e = copy_on(ctx->s, host, p, (size_t)ctx->ncell * 4, hipMemcpyDeviceToHost);
  return check_hip(ctx, e, "get_counts");
}

int itokmc_set_counts(itokmc_ctx* ctx, int which, const uint32_t* host) {
  if (!ctx || !host) return ITOKMC_EINVAL;
  uint32_t* p = counts_ptr(ctx, which);
  if (!p) return set_error(ctx, ITOKMC_EINVAL, "bad count selector");
  hipError_t e = hipStreamSynchronize(ctx->s);
  if (e == hipSuccess) e = copy_on(ctx->s, p, host, (size_t)ctx->ncell * 4, hipMemcpyHostToDevice);
  ctx->field_valid = false;
  return check_hip(ctx, e, "set_counts");
}

int itokmc_get_field(itokmc_ctx* ctx, double* phi) {
  if (!ctx || !phi) return ITOKMC_EINVAL;
  if (ctx->d.field_mode != ITOKMC_FIELD_POISSON) return set_error(ctx, ITOKMC_EINVAL, "uniform mode");
  return field_get_phi(ctx, phi);
}

int itokmc_set_field(itokmc_ctx* ctx, const double* phi) {
  if (!ctx || !phi) return ITOKMC_EINVAL;
  if (ctx->d.field_mode != ITOKMC_FIELD_POISSON) return set_error(ctx, ITOKMC_EINVAL, "uniform mode");
  return field_set_phi(ctx, phi);
}

int itokmc_set_tuning(itokmc_ctx* ctx, const itokmc_tuning* t) {
  if (!ctx || !t) return ITOKMC_EINVAL;
  if (t->mg_pre < 0 || t->mg_pre > 8 || t->mg_post < 0 || t->mg_post > 8 || t->mg_pre + t->mg_post < 1 ||
      t->bottom_sweeps < 0 || t->bottom_sweeps > 4096 || t->fine_layout < 0 || t->fine_layout > 1)
    return set_error(ctx, ITOKMC_EINVAL, "invalid tuning");
  ctx->tune = *t;
  field_reset_graph(ctx);
  return ITOKMC_OK;
}

int itokmc_get_tuning(itokmc_ctx* ctx, itokmc_tuning* t) {
  if (!ctx || !t) return ITOKMC_EINVAL;
  *t = ctx->tune;
  return ITOKMC_OK;
}

int itokmc_set_profiling(itokmc_ctx* ctx, int on) {
  if (!ctx) return ITOKMC_EINVAL;
  phase_collect(ctx);
  ctx->profiling = on != 0;
  if (ctx->d.field_mode == ITOKMC_FIELD_POISSON) field_set_timing(ctx, ctx->profiling);
  return ITOKMC_OK;
}

int itokmc_phase_times(itokmc_ctx* ctx, double* ms, uint64_t* calls, int n, int reset) {
  if (!ctx || !ms || !calls || n < 0) return ITOKMC_EINVAL;
  phase_collect(ctx);
  for (int i = 0; i < n && i < PH_NUM; ++i) {
    ms[i] = ctx->phase_ms[i];
    calls[i] = ctx->phase_calls[i];
  }
  if (reset)
    for (int i = 0; i < PH_NUM; ++i) { ctx->phase_ms[i] = 0.0; ctx->phase_calls[i] = 0; }
  return ITOKMC_OK;
}

void itokmc_destroy(itokmc_ctx* ctx) {
  if (!ctx) return;
  hipStreamSynchronize(ctx->s);
  for (auto& u : ctx->ev_used) { hipEventDestroy(u.second.first); hipEventDestroy(u.second.second); }
  for (auto e : ctx->ev_free) hipEventDestroy(e);
  field_destroy(ctx);
  if (ctx->host_ctr) (void)hipHostFree(ctx->host_ctr);
  delete ctx;
}

const char* itokmc_last_error(const itokmc_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int itokmc_philox_fill(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                       uint64_t n, uint32_t* dev_out, void* stream) {
  if (!dev_out && n) return ITOKMC_EINVAL;
  if (n == 0) return ITOKMC_OK;
  hipError_t e = launch_philox_fill(c0, c1, c2, c3, k0, k1, n, dev_out, (hipStream_t)stream);
  return e == hipSuccess ? ITOKMC_OK : ITOKMC_EHIP;
}

int itokmc_kmc_cells(itokmc_ctx* ctx, uint64_t n, const uint32_t* ids, int64_t* X, const double* k,
                     double dt, uint32_t step, int64_t* fires) {
  if (!ctx || (n && (!ids || !X || !k || !fires))) return ITOKMC_EINVAL;
  if (!(dt > 0.0)) return set_error(ctx, ITOKMC_EINVAL, "dt must be positive");
  if (n == 0) return ITOKMC_OK;
  return check_hip(ctx, launch_kmc_cells(ctx, n, ids, X, k, dt, step, fires), "kmc_cells");
}

int itokmc_rates(const itokmc_coeffs* c, double E, double dx, double* out) {
  std::string why;
  if (!c || !out || !(E >= 0.0) || !(dx > 0.0) || check_coeffs(c, &why)) return ITOKMC_EINVAL;
  const double mu = mobility(*c, E);
  const double alpha = E > 0.0 ? c->alpha_A * exp(-c->alpha_B / E) : 0.0;
  const double v = mu * E;
  out[0] = alpha * v;
  out[1] = c->eta * v;
  out[2] = c->kgamma_ratio * out[0];
  recomb_rates(*c, E, dx, out + 3);
  return ITOKMC_OK;
}

int itokmc_kmc_run(itokmc_ctx* ctx, uint64_t n, const uint32_t* ids, const uint32_t* real,
                   const uint32_t* nst, int64_t* X, const double* k, double dt, uint32_t step0,
                   uint32_t nsteps, int64_t* fires) {
  if (!ctx || (n && (!ids || !X || !k || !fires))) return ITOKMC_EINVAL;
  if (!(dt > 0.0)) return set_error(ctx, ITOKMC_EINVAL, "dt must be positive");
  if ((uint64_t)step0 + nsteps > 0x100000000ull)
    return set_error(ctx, ITOKMC_EINVAL, "step0 + nsteps exceeds the 32-bit step counter");
  if (n == 0 || (nsteps == 0 && !nst)) return ITOKMC_OK;
  return check_hip(ctx, launch_kmc_run(ctx, n, ids, real, nst, X, k, dt, step0, nsteps, fires), "kmc_run");
}

}  // extern "C"
