/*
 * Oracle random numbers (test infrastructure; see oracle.h).
 *
 * The paper leaves the generator unspecified: it needs uniform numbers for the SSA
 * (section "Stochastic simulation algorithm (SSA) and tau-leaping"), normal deviates
 * for the Ito kernel (eq. ito / ito_kernel), Poisson deviates for tau-leaping
 * (eq. tau_leaping) and uniform/exponential numbers for photon transport
 * (eq. photon_transport).  This file implements, from their published definitions:
 *   - Philox4x32-10, Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy
 *     as 1, 2, 3", SC'11: ten rounds of two 32x32->64 multiplies with the multipliers
 *     0xD2511F53, 0xCD9E8D57 and Weyl key increments 0x9E3779B9, 0xBB67AE85;
 *   - the Box-Muller transform (Box and Muller, 1958);
 *   - Poisson deviates by sequential CDF inversion for small means and by the
 *     transformed-rejection method PTRS of Hormann (1993) for means >= 10.
 * Pins: statistical tests (uniformity, normality, Poisson pmf); the generator words
 * against a third implementation, PyTorch's header-only CPU Philox engine, compiled
 * on the host by the tests (every counter and key word, 206 blocks).
 */
#include "or_internal.h"
#include <math.h>

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* uniform in [0,1) with 32-bit resolution */
double or_u_co(uint32_t x) { return (double)x * 0x1p-32; }
/* uniform in (0,1] with 32-bit resolution; used wherever a logarithm is taken */
double or_u_oc(uint32_t x) { return ((double)x + 1.0) * 0x1p-32; }
/* uniform in [0,1) with 24-bit resolution; used for positions inside a cell so that
 * the value is exactly representable in single precision */
double or_u24(uint32_t x) { return (double)(x >> 8) * 0x1p-24; }

void or_block(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t tag, uint32_t sub,
              uint32_t seed, uint32_t realization, uint32_t out[4]) {
  uint32_t ctr[4] = {c0, c1, c2, (tag << 24) | (sub & 0xFFFFFFu)};
  uint32_t key[2] = {seed, realization};
  or_philox4x32_10(ctr, key, out);
}

void or_stream_init(or_stream* s, uint32_t cell, uint32_t step, uint32_t tag, uint32_t sub,
                    uint32_t seed, uint32_t realization) {
  s->cell = cell; s->step = step; s->tag = tag; s->sub = sub;
  s->seed = seed; s->realization = realization;
  s->n = 0;
}

/* Word n of a cell's sequential stream is word (n mod 4) of the Philox block with
 * counter (cell, n div 4, step, tag|sub). */
uint32_t or_stream_next(or_stream* s) {
  uint32_t blk = s->n >> 2, lane = s->n & 3u;
  if (lane == 0)
    or_block(s->cell, blk, s->step, s->tag, s->sub, s->seed, s->realization, s->buf);
  s->n++;
  return s->buf[lane];
}

void or_normals3(uint64_t id, uint32_t step, uint32_t seed, uint32_t realization,
                 double out[3]) {
  uint32_t x[4];
  or_block((uint32_t)id, (uint32_t)(id >> 32), step, OR_TAG_PUSH, 0, seed, realization, x);
  const double two_pi = 6.283185307179586476925286766559;
  double r0 = sqrt(-2.0 * log(or_u_oc(x[0])));
  double t0 = two_pi * or_u_co(x[1]);
  double r1 = sqrt(-2.0 * log(or_u_oc(x[2])));
  double t1 = two_pi * or_u_co(x[3]);
  out[0] = r0 * cos(t0);
  out[1] = r0 * sin(t0);
  out[2] = r1 * cos(t1);
}

/* Poisson deviate with mean lambda drawn from the stream s.
 *   lambda <= 0 : 0, no draw;
 *   lambda < 10 : one uniform u in [0,1); smallest k with F(k) > u, F the Poisson CDF
 *                 accumulated term by term;
 *   otherwise   : PTRS (Hormann 1993), two uniforms per trial. */
int64_t or_poisson(double lambda, or_stream* s) {
  if (!(lambda > 0.0)) return 0;
  if (lambda < 10.0) {
    double u = or_u_co(or_stream_next(s));
    double p = exp(-lambda);
    double F = p;
    int64_t k = 0;
    while (u >= F && k < 1000) {
      k += 1;
      p *= lambda / (double)k;
      F += p;
    }
    return k;
  }
  double slam = sqrt(lambda);
  double loglam = log(lambda);
  double b = 0.931 + 2.53 * slam;
  double a = -0.059 + 0.02483 * b;
  double inv_alpha = 1.1239 + 1.1328 / (b - 3.4);
  double v_r = 0.9277 - 3.6224 / (b - 2.0);
  for (;;) {
    double U = or_u_co(or_stream_next(s)) - 0.5;
    double V = or_u_oc(or_stream_next(s));
    double us = 0.5 - fabs(U);
    double kd = floor((2.0 * a / us + b) * U + lambda + 0.43);
    if (us >= 0.07 && V <= v_r) return (int64_t)kd;
    if (kd < 0.0 || (us < 0.013 && V > us)) continue;
    double lhs = log(V) + log(inv_alpha) - log(a / (us * us) + b);
    double rhs = -lambda + kd * loglam - lgamma(kd + 1.0);
    if (lhs <= rhs) return (int64_t)kd;
  }
}

int64_t or_poisson_draw(double lambda, uint32_t cell, uint32_t step, uint32_t seed,
                        uint32_t realization, uint32_t* n_used) {
  or_stream s;
  or_stream_init(&s, cell, step, OR_TAG_KMC, 0, seed, realization);
  int64_t k = or_poisson(lambda, &s);
  if (n_used) *n_used = s.n;
  return k;
}
