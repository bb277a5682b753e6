/* Oracle internals (test infrastructure; see oracle.h). */
#ifndef ITOKMC_OR_INTERNAL_H
#define ITOKMC_OR_INTERNAL_H
#include "oracle.h"
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define OR_E_CHARGE 1.602176634e-19 /* C */
#define OR_EPS0 8.8541878128e-12    /* F/m */

typedef struct {
  uint32_t cell, step, tag, sub, seed, realization;
  uint32_t n;      /* words consumed */
  uint32_t buf[4];
} or_stream;

typedef struct {
  double xi[3];    /* position in grid units */
  uint64_t w;
  uint64_t id;
} or_particle;

struct or_sim {
  or_desc d;
  or_coeffs c;
  int64_t ncell;
  uint64_t cap, np;
  or_particle* p;
  int64_t *nplus, *nminus, *ngamma;
  int64_t* fires;              /* 3 per cell, last react phase */
  double *phi, *Ex, *Ey, *Ez;  /* Poisson mode */
  int field_valid;
  uint32_t step;
  or_diag diag;
};

double or_u_co(uint32_t x);
double or_u_oc(uint32_t x);
double or_u24(uint32_t x);
void or_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, uint32_t sub,
              uint32_t seed, uint32_t realization, uint32_t out[4]);
void or_stream_init(or_stream* s, uint32_t cell, uint32_t step, uint32_t tag, uint32_t sub,
                    uint32_t seed, uint32_t realization);
uint32_t or_stream_next(or_stream* s);
int64_t or_poisson(double lambda, or_stream* s);

/* KMC on one cell: X[4] in/out, k[5], returns fires[5] */
void or_kmc_advance(const or_desc* d, int64_t X[4], const double k[5], double dt,
                    or_stream* s, int64_t fires[5]);

uint64_t or_make_id(int kind, uint32_t step, uint32_t cell, uint32_t slot);
/* split N physical particles into at most n_new computational ones: returns M,
 * weight of slot s is w_base (+ remainder for s == 0) */
int32_t or_split_count(int64_t N, int32_t n_new, int64_t* w_base, int64_t* w_rem);

/* particle store */
int or_push_particle(or_sim* s, const double xi[3], uint64_t w, uint64_t id);
int64_t or_cell_of(const or_desc* d, const double xi[3]); /* -1 if outside */

#endif
