/*
 * Oracle: field solve and cloud-in-cell transfer (test infrastructure; see oracle.h).
 *
 * Field: the semi-implicit Poisson equation of the paper's section "Semi-implicit
 * Euler-Maruyama method" (eqs. poisson_simp and conductivity),
 *     div[(1 + sigma dt / eps0) grad phi] = -rho / eps0,   E = -grad phi,
 * discretised by finite volumes on the uniform grid: a 7-point stencil with face
 * coefficients equal to the harmonic mean of the two adjacent cell values, phi = 0 on
 * the face z = 0, phi = V_anode on z = L (a Dirichlet face uses the cell's own
 * coefficient over half a cell), homogeneous Neumann on the x and y faces.  The
 * paper solves this with geometric multigrid to a relative tolerance of 1e-10; the
 * oracle solves the same linear system by plain conjugate gradients (the operator is
 * symmetric positive definite), to a tighter tolerance, so that it defines the
 * discrete solution rather than an approximation of it.  E at a cell centre is the
 * central difference of phi with ghost values from the same boundary conditions.
 *
 * CIC: eq. for n_i with the tent kernel W_cic of the section "Charge deposition &
 * interpolation", with cell centres at (i + 1/2) dx.  The part of a cloud that lies
 * beyond the outermost cell centres is folded back into the wall cell (the paper's
 * embedded boundaries do not exist here), which conserves the deposited total;
 * interpolation uses the same weights.  A workload may select the quadratic B-spline
 * (TSC) shape instead (or_tsc_*, below), with the same conventions.
 * Pins (tests): rho = 0 gives the linear potential and the uniform field V/L;
 * manufactured solutions converge at second order; a constant coefficient scales
 * the solution; single-particle CIC weights; total deposited weight.
 */
#include "or_internal.h"

static inline int64_t IDX(const or_desc* d, int i, int j, int k) {
  return (int64_t)i + (int64_t)d->nx * ((int64_t)j + (int64_t)d->ny * k);
}

static double hmean(double a, double b) { return 2.0 * a * b / (a + b); }

/* y = A x for the homogeneous operator (boundary values zero), scaled by dx^2 */
static void apply_A(const or_desc* d, const double* eps, const double* x, double* y) {
  int nx = d->nx, ny = d->ny, nz = d->nz;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t c = IDX(d, i, j, k);
        double ec = eps[c], xc = x[c], acc = 0.0;
        if (i > 0) { int64_t n = IDX(d, i - 1, j, k); acc += hmean(ec, eps[n]) * (xc - x[n]); }
        if (i < nx - 1) { int64_t n = IDX(d, i + 1, j, k); acc += hmean(ec, eps[n]) * (xc - x[n]); }
        if (j > 0) { int64_t n = IDX(d, i, j - 1, k); acc += hmean(ec, eps[n]) * (xc - x[n]); }
        if (j < ny - 1) { int64_t n = IDX(d, i, j + 1, k); acc += hmean(ec, eps[n]) * (xc - x[n]); }
        if (k > 0) { int64_t n = IDX(d, i, j, k - 1); acc += hmean(ec, eps[n]) * (xc - x[n]); }
        else acc += 2.0 * ec * xc;
        if (k < nz - 1) { int64_t n = IDX(d, i, j, k + 1); acc += hmean(ec, eps[n]) * (xc - x[n]); }
        else acc += 2.0 * ec * xc;
        y[c] = acc;
      }
}

static double dot(int64_t n, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

int or_solve_poisson(const or_desc* d, const double* rho, const double* eps_r, double* phi,
                     double rtol, int max_iter, double* relres) {
  int64_t n = (int64_t)d->nx * d->ny * d->nz;
  double h2 = d->dx * d->dx;
  double* b = (double*)malloc(sizeof(double) * (size_t)n);
  double* r = (double*)malloc(sizeof(double) * (size_t)n);
  double* p = (double*)malloc(sizeof(double) * (size_t)n);
  double* Ap = (double*)malloc(sizeof(double) * (size_t)n);
  /* right-hand side scaled by dx^2, including the Dirichlet lift on z = L */
  for (int k = 0; k < d->nz; ++k)
    for (int j = 0; j < d->ny; ++j)
      for (int i = 0; i < d->nx; ++i) {
        int64_t c = IDX(d, i, j, k);
        b[c] = h2 * rho[c] / OR_EPS0;
        if (k == d->nz - 1) b[c] += 2.0 * eps_r[c] * d->V_anode;
      }
  double bnorm = sqrt(dot(n, b, b));
  apply_A(d, eps_r, phi, Ap);
  for (int64_t i = 0; i < n; ++i) { r[i] = b[i] - Ap[i]; p[i] = r[i]; }
  double rr = dot(n, r, r);
  int it = 0;
  if (bnorm == 0.0) bnorm = 1.0;
  while (sqrt(rr) > rtol * bnorm && it < max_iter) {
    apply_A(d, eps_r, p, Ap);
    double alpha = rr / dot(n, p, Ap);
    for (int64_t i = 0; i < n; ++i) { phi[i] += alpha * p[i]; r[i] -= alpha * Ap[i]; }
    double rr2 = dot(n, r, r);
    double beta = rr2 / rr;
    for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
    rr = rr2;
    ++it;
  }
  /* report the true residual */
  apply_A(d, eps_r, phi, Ap);
  double tr = 0.0;
  for (int64_t i = 0; i < n; ++i) { double e = b[i] - Ap[i]; tr += e * e; }
  if (relres) *relres = sqrt(tr) / bnorm;
  free(b); free(r); free(p); free(Ap);
  return it;
}

/* ||b - A phi||_2 / ||b||_2 of the system or_solve_poisson solves (same b, same A). */
double or_poisson_relres(const or_desc* d, const double* rho, const double* eps_r,
                         const double* phi) {
  int64_t n = (int64_t)d->nx * d->ny * d->nz;
  double h2 = d->dx * d->dx;
  double* Ap = (double*)malloc(sizeof(double) * (size_t)n);
  apply_A(d, eps_r, phi, Ap);
  double bb = 0.0, rr = 0.0;
  for (int k = 0; k < d->nz; ++k)
    for (int j = 0; j < d->ny; ++j)
      for (int i = 0; i < d->nx; ++i) {
        int64_t c = IDX(d, i, j, k);
        double b = h2 * rho[c] / OR_EPS0;
        if (k == d->nz - 1) b += 2.0 * eps_r[c] * d->V_anode;
        bb += b * b;
        rr += (b - Ap[c]) * (b - Ap[c]);
      }
  free(Ap);
  return bb > 0.0 ? sqrt(rr / bb) : sqrt(rr);
}

void or_efield(const or_desc* d, const double* phi, double* Ex, double* Ey, double* Ez) {
  int nx = d->nx, ny = d->ny, nz = d->nz;
  double inv2h = 1.0 / (2.0 * d->dx);
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        int64_t c = IDX(d, i, j, k);
        double pc = phi[c];
        double xm = i > 0 ? phi[IDX(d, i - 1, j, k)] : pc;           /* Neumann ghost */
        double xp = i < nx - 1 ? phi[IDX(d, i + 1, j, k)] : pc;
        double ym = j > 0 ? phi[IDX(d, i, j - 1, k)] : pc;
        double yp = j < ny - 1 ? phi[IDX(d, i, j + 1, k)] : pc;
        double zm = k > 0 ? phi[IDX(d, i, j, k - 1)] : -pc;          /* phi = 0 at z = 0 */
        double zp = k < nz - 1 ? phi[IDX(d, i, j, k + 1)] : 2.0 * d->V_anode - pc;
        Ex[c] = -(xp - xm) * inv2h;
        Ey[c] = -(yp - ym) * inv2h;
        Ez[c] = -(zp - zm) * inv2h;
      }
}

/* clamped tent weights along one axis: lower node index and weight of upper node */
static void cic_axis(double xi, int n, int* i0, double* f) {
  double s = xi - 0.5;
  if (s < 0.0) s = 0.0;
  if (s > (double)(n - 1)) s = (double)(n - 1);
  if (n == 1) { *i0 = 0; *f = 0.0; return; }
  int i = (int)floor(s);
  if (i > n - 2) i = n - 2;
  *i0 = i;
  *f = s - (double)i;
}

void or_cic_deposit(const or_desc* d, uint64_t n, const double* xi, const double* q,
                    double* grid) {
  for (uint64_t p = 0; p < n; ++p) {
    int i0, j0, k0;
    double fx, fy, fz;
    cic_axis(xi[3 * p + 0], d->nx, &i0, &fx);
    cic_axis(xi[3 * p + 1], d->ny, &j0, &fy);
    cic_axis(xi[3 * p + 2], d->nz, &k0, &fz);
    for (int c = 0; c < 8; ++c) {
      int di = c & 1, dj = (c >> 1) & 1, dk = (c >> 2) & 1;
      double wgt = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
      if (wgt == 0.0) continue;
      int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
      if (ii >= d->nx || jj >= d->ny || kk >= d->nz) continue; /* only when n == 1 */
      grid[IDX(d, ii, jj, kk)] += q[p] * wgt;
    }
  }
}

void or_cic_interp(const or_desc* d, const double* grid, uint64_t n, const double* xi,
                   double* out) {
  for (uint64_t p = 0; p < n; ++p) {
    int i0, j0, k0;
    double fx, fy, fz;
    cic_axis(xi[3 * p + 0], d->nx, &i0, &fx);
    cic_axis(xi[3 * p + 1], d->ny, &j0, &fy);
    cic_axis(xi[3 * p + 2], d->nz, &k0, &fz);
    double acc = 0.0;
    for (int c = 0; c < 8; ++c) {
      int di = c & 1, dj = (c >> 1) & 1, dk = (c >> 2) & 1;
      double wgt = (di ? fx : 1.0 - fx) * (dj ? fy : 1.0 - fy) * (dk ? fz : 1.0 - fz);
      if (wgt == 0.0) continue;
      int ii = i0 + di, jj = j0 + dj, kk = k0 + dk;
      if (ii >= d->nx || jj >= d->ny || kk >= d->nz) continue;
      acc += grid[IDX(d, ii, jj, kk)] * wgt;
    }
    out[p] = acc;
  }
}

/* TSC: the quadratic B-spline cloud (a unit box convolved with the CIC tent), one of
 * the higher-order particle shapes the paper's future-work section points to.  Along an
 * axis with cell centres at j + 1/2, a particle at xi has its nearest centre j =
 * floor(xi), offset d = xi - j - 1/2 in [-1/2, 1/2), and weights (1/2 - d)^2 / 2,
 * 3/4 - d^2 and (1/2 + d)^2 / 2 on the centres j - 1, j, j + 1.  A centre outside the
 * grid hands its weight to the wall cell (clamped index), which conserves the total and
 * keeps the weights a convex combination; interpolation uses the same weights.  Its
 * moments pin it: the weights sum to 1, reproduce xi as the first moment and xi^2 + 1/4
 * as the second (inside the grid), and equal the CIC weights averaged over a unit box
 * centred on the particle. */
static void tsc_axis(double xi, int n, int idx[3], double w[3]) {
  const double j = floor(xi);
  const double dd = xi - j - 0.5;
  w[0] = 0.5 * (0.5 - dd) * (0.5 - dd);
  w[1] = 0.75 - dd * dd;
  w[2] = 0.5 * (0.5 + dd) * (0.5 + dd);
  for (int a = 0; a < 3; ++a) {
    double t = j - 1.0 + (double)a;
    if (t < 0.0) t = 0.0;
    if (t > (double)(n - 1)) t = (double)(n - 1);
    idx[a] = (int)t;
  }
}

void or_tsc_deposit(const or_desc* d, uint64_t n, const double* xi, const double* q,
                    double* grid) {
  for (uint64_t p = 0; p < n; ++p) {
    int ix[3], iy[3], iz[3];
    double wx[3], wy[3], wz[3];
    tsc_axis(xi[3 * p + 0], d->nx, ix, wx);
    tsc_axis(xi[3 * p + 1], d->ny, iy, wy);
    tsc_axis(xi[3 * p + 2], d->nz, iz, wz);
    for (int c = 0; c < 3; ++c)
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          double wgt = wx[a] * wy[b] * wz[c];
          if (wgt == 0.0) continue;
          grid[IDX(d, ix[a], iy[b], iz[c])] += q[p] * wgt;
        }
  }
}

void or_tsc_interp(const or_desc* d, const double* grid, uint64_t n, const double* xi,
                   double* out) {
  for (uint64_t p = 0; p < n; ++p) {
    int ix[3], iy[3], iz[3];
    double wx[3], wy[3], wz[3];
    tsc_axis(xi[3 * p + 0], d->nx, ix, wx);
    tsc_axis(xi[3 * p + 1], d->ny, iy, wy);
    tsc_axis(xi[3 * p + 2], d->nz, iz, wz);
    double acc = 0.0;
    for (int c = 0; c < 3; ++c)
      for (int b = 0; b < 3; ++b)
        for (int a = 0; a < 3; ++a) {
          double wgt = wx[a] * wy[b] * wz[c];
          if (wgt == 0.0) continue;
          acc += grid[IDX(d, ix[a], iy[b], iz[c])] * wgt;
        }
    out[p] = acc;
  }
}

void or_cloud_deposit(const or_desc* d, uint64_t n, const double* xi, const double* q,
                      double* grid) {
  if (d->shape == OR_SHAPE_TSC) or_tsc_deposit(d, n, xi, q, grid);
  else or_cic_deposit(d, n, xi, q, grid);
}

void or_cloud_interp(const or_desc* d, const double* grid, uint64_t n, const double* xi,
                     double* out) {
  if (d->shape == OR_SHAPE_TSC) or_tsc_interp(d, grid, n, xi, out);
  else or_cic_interp(d, grid, n, xi, out);
}
