// Internal context of the itokmc library (host side) and kernel launcher prototypes.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

#include "../../include/itokmc.h"

namespace itk {
// Host copies of the library go through the context's stream and wait for it: never the
// legacy default stream, which the runtime forbids while any other thread captures a
// stream into a graph.
inline hipError_t copy_on(hipStream_t s, void* dst, const void* src, size_t bytes, hipMemcpyKind kind) {
  hipError_t e = hipMemcpyAsync(dst, src, bytes, kind, s);
  return e == hipSuccess ? hipStreamSynchronize(s) : e;
}

// Structure-of-arrays particle bank.  Offsets are cell-relative in [0,1) and stored
// in the working precision (float or double) as three separate arrays so that each
// lane's loads coalesce.
struct Bank {
  uint32_t* cell;
  void* ox;
  void* oy;
  void* oz;
  uint32_t* w;
  uint64_t* id;
  uint32_t* rank;  // position inside the destination cell, written by the push
};

// Device-resident counters and tallies (one 256-byte block of the arena).
struct Counters {
  uint32_t n[2];          // particles per bank (including dead slots, w == 0)
  uint32_t overflow;      // ITOKMC_OVF_*: bit 0 particle capacity, bit 1 a cell too
                          // large for every merge staging (left unmerged)
  uint32_t n_occ;         // occupied cells after binning
  uint32_t n_work;        // cells needing coupling / merge
  uint32_t sorted;        // particles placed by the last counting sort
  uint32_t n_heavy;       // occupied cells left to the full KMC pass
  uint32_t n_huge;        // cells deferred past the mid-size merge staging
  unsigned long long outflow, created, removed, merged;
  unsigned long long fires[5];  // ionization, attachment, emission, e-ion, ion-ion
  unsigned long long ph_emitted, ph_absorbed, ph_lost;
  unsigned long long pushed;   // live particles advanced by the transport kernels
  uint32_t merge_skipped;      // cells too large for the LDS merge (left unmerged)
  uint32_t n_big;              // cells deferred to the mid-size merge staging
  uint32_t n_cfull;            // cells for the wavefront coupling pass (everything)
  uint32_t n_cmerge;           // cells for the wavefront coupling pass (merge only)
  unsigned long long couple_pieces;  // particles gathered by the wavefront coupling pass
  // device-side stop rule (itokmc_step_until): once halt is set, every kernel of the
  // step path returns at entry, so the state stays that of the last step taken
  uint32_t halt;
  uint32_t steps_done;
  unsigned long long pushed_mark;    // `pushed` at the start of the current step
  unsigned long long ion_out[2];     // positive and negative ions lost through domain faces
  uint32_t n_ionbig;                 // ion species of large total mean left to the second pass
  uint32_t pad_ion;
};

// Device-side copy of the per-step constants shared by the kernels.
struct StepConst {
  int nx, ny, nz;
  uint32_t ncell;
  uint32_t cap;
  uint32_t step;
  Key key;
  double dx, dt;
  double drift[3];   // uniform mode: -mu E dt / dx per axis (grid units)
  double diff;       // sqrt(2 D dt) / dx (grid units per unit normal)
  double k[5];       // uniform mode rates (1/s): k_alpha, k_eta, k_gamma, k_ep, k_np
  // multiply-shift division by nx and by ny: floor(c / d) = (c * m) >> s for every
  // c < 2^24, with s = 24 + ceil(log2 d) and m = ceil(2^s / d) (< 2^25)
  uint32_t mdx, sdx, mdy, sdy;
};

// Cell indices (i, j, k) of a cell number c = i + nx (j + ny k), by multiply-shift
// division (StepConst.mdx/sdx/mdy/sdy).
__device__ __forceinline__ void cell_ijk(uint32_t c, const StepConst& K, int& i, int& j, int& k) {
  const uint32_t row = (uint32_t)(((uint64_t)c * K.mdx) >> K.sdx);
  i = (int)(c - row * (uint32_t)K.nx);
  const uint32_t kk = (uint32_t)(((uint64_t)row * K.mdy) >> K.sdy);
  j = (int)(row - kk * (uint32_t)K.ny);
  k = (int)kk;
}
// Host: the multiply-shift constants of a divisor d in [1, 2^24].
inline void div_magic(uint32_t d, uint32_t* m, uint32_t* s) {
  uint32_t l = 0;
  while ((1u << l) < d) ++l;
  *s = 24 + l;
  *m = (uint32_t)(((1ull << *s) + d - 1) / d);
}

// Field view for per-cell KMC rates (Poisson mode): E at cell centres, packed
// (Ex, Ey, Ez, 0) per cell, and the coefficient forms; E4 == nullptr means the
// prescribed uniform field.
struct FieldRates {
  const void* E4;
  int is_double;
  double mu_a, mu_E0, mu_b, E_floor, alpha_A, alpha_B, eta, kgamma_ratio;
  double beta_ep, beta_ep_b, Te_a, Te_b, beta_np, dV;  // recombination (0: off)
};

}  // namespace itk

struct itokmc_ctx {
  itokmc_grid_desc d;
  itokmc_coeffs c;
  bool have_coeffs = false;
  hipStream_t s = nullptr;
  char* arena = nullptr;
  size_t arena_bytes = 0;
  uint32_t ncell = 0;
  uint64_t cap = 0;
  int cur = 0;  // bank holding the current particles
  itk::Bank bank[2];
  // per-cell arrays
  unsigned long long* cellacc = nullptr;  // (count << 32) | weight, reset after use
  uint32_t* start = nullptr;              // ncell + 1 exclusive prefix of counts
  uint32_t* occ = nullptr;                // occupied cells (n_occ entries)
  uint32_t* occ_fires = nullptr;          // 3 per occupied cell: fires of the last step
  uint32_t* nplus = nullptr;
  uint32_t* nminus = nullptr;
  uint32_t* ngamma = nullptr;
  int32_t* dN = nullptr;                  // net electron change per occupied cell
  uint32_t* work = nullptr;               // occupied-cell indices needing coupling
  uint32_t* cbase = nullptr;              // first reserved bank slot of a cell's products
  uint32_t* big = nullptr;                // occupied-cell indices for the mid-size merge pass
  uint32_t* huge = nullptr;               // occupied-cell indices for the large merge pass
  uint32_t* cfull = nullptr;              // cells for the wavefront coupling pass
  uint32_t* cmerge = nullptr;             // cells to merge after the light coupling pass
  uint32_t* ion_next[2] = {nullptr, nullptr};  // ion counts after a transport move (M+, M-)
  uint32_t* ion_big = nullptr;            // (cell << 1 | species) of large total mean, 2 ncell
  void* mu_p = nullptr;                   // per particle (self-consistent mode): mu(|E^k(X^k)|)
                                          // written by the deposit, read by the push
  uint32_t* heavy = nullptr;              // occupied-cell indices for the full KMC pass
  double* rates = nullptr;                // 3 per occupied cell: rates handed to the full pass
  uint32_t* blocksums = nullptr;          // scan scratch
  uint32_t* tiles = nullptr;               // per 2048-cell tile: received particles
  itk::Counters* ctr = nullptr;
  unsigned long long* reduce = nullptr;   // small reduction scratch
  bool binned = false;                    // bins of the current bank are filled
  itk::Counters* host_ctr = nullptr;      // pinned mirror
  // Poisson-mode field data (see field.hip)
  void* field = nullptr;        // arena region
  void* field_state = nullptr;  // host-side bookkeeping (FieldState)
  bool field_valid = false;
  int last_cycles = 0;
  uint64_t total_cycles = 0;   // multigrid cycles over all solves
  uint64_t total_solves = 0;
  double last_relres = 0.0;
  uint32_t step = 0;
  std::string err;
  // optional per-phase timing with HIP events recorded on the context's stream
  bool profiling = false;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_used;
  std::vector<hipEvent_t> ev_free;
  double phase_ms[16] = {0};      // indexed by itk::Phase (< 16)
  uint64_t phase_calls[16] = {0};
  itokmc_tuning tune = {2, 2, 0, 1, 1, 0};
};

namespace itk {
// phases timed when profiling is on
enum Phase { PH_PUSH = 0, PH_PHOTON, PH_SCAN, PH_SCATTER, PH_KMC, PH_COUPLE, PH_DEPOSIT,
             PH_SOLVE, PH_FIELD_PUSH, PH_COUNT, PH_MERGE, PH_FIELD_PREP, PH_SMOOTH_FINE,
             PH_COUPLE_LIGHT, PH_EMAX, PH_IONS, PH_NUM };
void phase_begin(itokmc_ctx* ctx, int phase);
void phase_end(itokmc_ctx* ctx, int phase);
int set_error(itokmc_ctx* ctx, int code, const char* fmt, ...);
int check_hip(itokmc_ctx* ctx, hipError_t e, const char* what);

StepConst make_const(const itokmc_ctx* ctx, double dt);
// Uniform-field drift and diffusion per step (grid units) and rates (1/s).
void uniform_consts(const itokmc_grid_desc& d, const itokmc_coeffs& c, double dt,
                    double drift[3], double* diff, double k[5]);
void recomb_rates(const itokmc_coeffs& c, double Em, double dx, double k[2]);
// Recombination (electron-ion or ion-ion) is part of the context's network.
inline bool recombination(const itokmc_ctx* ctx) {
  return ctx->c.beta_ep > 0.0 || ctx->c.beta_np > 0.0;
}
bool valid_desc(const itokmc_grid_desc* d);
int check_coeffs(const itokmc_coeffs* c, std::string* why);
// particles.hip
hipError_t launch_seed_gaussian(itokmc_ctx* ctx, const itokmc_seed_desc* sd);
hipError_t launch_seed_neutral(itokmc_ctx* ctx, const itokmc_seed_desc* sd);
hipError_t launch_push_uniform(itokmc_ctx* ctx, const StepConst& k);
hipError_t launch_count(itokmc_ctx* ctx);  // bin the current bank without moving
hipError_t launch_photons(itokmc_ctx* ctx, const StepConst& k);
hipError_t launch_scan(itokmc_ctx* ctx);
hipError_t launch_scatter(itokmc_ctx* ctx);
// pointer forms used by the ensemble (ncell_dev: device-side cell count to scan)
hipError_t launch_scan_raw(const unsigned long long* cellacc, uint32_t max_cells,
                           const uint32_t* ncell_dev, uint32_t* tiles, uint32_t* blocksums,
                           uint32_t* start, uint32_t* occ, Counters* ctr, int dest, hipStream_t s);
// u32 words of scan scratch for a cell count
size_t scan_scratch_words(uint64_t ncell);
hipError_t launch_scatter_raw(Bank a, Bank b, Counters* ctr, int which, const uint32_t* start,
                              uint32_t cap, int fp64, int grid, hipStream_t s);
hipError_t launch_ngp(itokmc_ctx* ctx, uint32_t* out);
hipError_t launch_reduce_particles(itokmc_ctx* ctx, unsigned long long* out2);
hipError_t launch_reduce_cells(itokmc_ctx* ctx, unsigned long long* out2);
hipError_t launch_fires_dense(itokmc_ctx* ctx, uint32_t* out);
hipError_t launch_philox_fill(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                              uint32_t k1, uint64_t n, uint32_t* out, hipStream_t s);
// kmc.hip
hipError_t launch_kmc_step(itokmc_ctx* ctx, const StepConst& k, const FieldRates& fr);
hipError_t launch_stop_begin(itokmc_ctx* ctx);
hipError_t launch_stop_step(itokmc_ctx* ctx, uint64_t stop_particles);
hipError_t launch_stop_end(itokmc_ctx* ctx);
hipError_t launch_kmc_run(itokmc_ctx* ctx, uint64_t n, const uint32_t* ids, const uint32_t* real,
                          const uint32_t* nst, int64_t* X, const double* k, double dt, uint32_t step0,
                          uint32_t nsteps, int64_t* fires);
hipError_t launch_kmc_cells(itokmc_ctx* ctx, uint64_t n, const uint32_t* ids, int64_t* X,
                            const double* k, double dt, uint32_t step, int64_t* fires);
// couple.hip
hipError_t launch_couple(itokmc_ctx* ctx, const StepConst& k);
// ions.hip: move the ion counts with the step's field (E4: packed cell-centre field of
// the precision's type, or null for the prescribed uniform field); no-op without ion
// transport coefficients
inline bool mobile_ions(const itokmc_ctx* ctx) { return ctx->c.mu_ion > 0.0 || ctx->c.D_ion > 0.0; }
hipError_t launch_ion_move(itokmc_ctx* ctx, const StepConst& k, const void* E4);
// field.hip (Poisson mode)
size_t field_bytes(const itokmc_grid_desc* d);
int field_init(itokmc_ctx* ctx, char* base);
int field_transport(itokmc_ctx* ctx, const StepConst& k);
// Largest |E| over the cell centres of E^k (computes the initial field if there is none).
int field_max(itokmc_ctx* ctx, double* Emax);
FieldRates field_rates(itokmc_ctx* ctx);  // E view for the KMC rates
void field_destroy(itokmc_ctx* ctx);
void field_reset_graph(itokmc_ctx* ctx);
void field_set_timing(itokmc_ctx* ctx, bool on);
int field_get_phi(itokmc_ctx* ctx, double* host);
int field_set_phi(itokmc_ctx* ctx, const double* host);
int field_deposit(itokmc_ctx* ctx, int what, void* dev_out);
hipError_t launch_cic_density(itokmc_ctx* ctx, double* out);
hipError_t launch_rho(itokmc_ctx* ctx, double* out);
}  // namespace itk
