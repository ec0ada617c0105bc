/*
 * synthgen: seeded synthetic inputs shared by the GPU path and the oracle.
 *
 * This module holds no arithmetic of the Dirac operator or of the solvers.  It
 * only turns (seed, index) pairs into random numbers and random group
 * elements:
 *
 *   - Philox-4x32-10, the counter-based generator of Salmon, Moraes, Dror and
 *     Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC11, 2011);
 *   - Box-Muller Gaussians from pairs of 53-bit uniforms;
 *   - SU(3) link variables U = exp(X), X a traceless anti-Hermitian matrix with
 *     Gaussian entries, evaluated by scaling and squaring of a Taylor series
 *     and then projected back onto SU(3) (Gram-Schmidt of the first two rows,
 *     third row = complex conjugate of their cross product);
 *   - U(1) angles A ~ N(0, sigma^2), not wrapped into [-pi, pi];
 *   - Gaussian complex spinors with Re, Im ~ N(0, 1/2), so E|eta_i|^2 = 1.
 *
 * Every value depends only on (seed, tag, index, component), so any subset of
 * sites can be regenerated on its own (that is what lets a test regenerate the
 * neighbourhood of a sampled site of a very large lattice).
 *
 * Complex numbers are stored as interleaved (re, im) doubles.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#define SG_TAG_SU3 1u
#define SG_TAG_U1 2u
#define SG_TAG_SPINOR 3u
#define SG_TAG_TRANSFORM 4u
#define SG_TAG_REAL 5u
#define SG_TAG_ANGLE 6u

/* ---- Philox-4x32-10 ---------------------------------------------------- */

static inline void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

void sg_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
  uint32_t k0 = key_in[0], k1 = key_in[1];
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, c0, &hi0, &lo0);
    mulhilo32(M1, c2, &hi1, &lo1);
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    k0 += W0;
    k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* One Philox block -> two standard normal deviates. */
static void gauss2(uint64_t seed, uint32_t tag, uint64_t index, uint32_t sub, double *g0, double *g1) {
  uint32_t ctr[4] = {(uint32_t)index, (uint32_t)(index >> 32), sub, tag};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32) ^ 0x5EEDu};
  uint32_t r[4];
  sg_philox4x32_10(ctr, key, r);
  const double two53 = 9007199254740992.0;
  double u0 = ((double)(((uint64_t)(r[0] >> 5) << 26) | (r[1] >> 6)) + 0.5) / two53;
  double u1 = ((double)(((uint64_t)(r[2] >> 5) << 26) | (r[3] >> 6)) + 0.5) / two53;
  double rad = sqrt(-2.0 * log(u0));
  double ang = 6.283185307179586476925286766559 * u1;
  *g0 = rad * cos(ang);
  *g1 = rad * sin(ang);
}

/* ---- 3x3 complex helpers (row-major, interleaved) ------------------------ */

typedef struct { double re, im; } cplx;

static void mat_mul(const cplx *a, const cplx *b, cplx *c) {
  cplx t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double re = 0, im = 0;
      for (int k = 0; k < 3; ++k) {
        re += a[3 * i + k].re * b[3 * k + j].re - a[3 * i + k].im * b[3 * k + j].im;
        im += a[3 * i + k].re * b[3 * k + j].im + a[3 * i + k].im * b[3 * k + j].re;
      }
      t[3 * i + j].re = re;
      t[3 * i + j].im = im;
    }
  memcpy(c, t, sizeof(t));
}

/* exp(X) by scaling and squaring, then projection onto SU(3). */
static void su3_exp(const cplx *x, cplx *u) {
  double nrm = 0;
  for (int i = 0; i < 9; ++i) nrm += x[i].re * x[i].re + x[i].im * x[i].im;
  nrm = sqrt(nrm);
  int s = 0;
  while (nrm > 0.25) { nrm *= 0.5; ++s; }
  double scale = ldexp(1.0, -s);
  cplx y[9], term[9], e[9];
  for (int i = 0; i < 9; ++i) { y[i].re = x[i].re * scale; y[i].im = x[i].im * scale; }
  for (int i = 0; i < 9; ++i) { e[i].re = (i % 4 == 0) ? 1.0 : 0.0; e[i].im = 0.0; term[i] = e[i]; }
  for (int k = 1; k <= 16; ++k) {
    mat_mul(term, y, term);
    for (int i = 0; i < 9; ++i) { term[i].re /= k; term[i].im /= k; }
    for (int i = 0; i < 9; ++i) { e[i].re += term[i].re; e[i].im += term[i].im; }
  }
  for (int i = 0; i < s; ++i) mat_mul(e, e, e);
  /* Gram-Schmidt of rows 0 and 1, row 2 = conj(row0 x row1): det = 1. */
  cplx *r0 = e, *r1 = e + 3;
  double n0 = 0;
  for (int i = 0; i < 3; ++i) n0 += r0[i].re * r0[i].re + r0[i].im * r0[i].im;
  n0 = 1.0 / sqrt(n0);
  for (int i = 0; i < 3; ++i) { r0[i].re *= n0; r0[i].im *= n0; }
  double pre = 0, pim = 0; /* <r0, r1> = sum conj(r0) r1 */
  for (int i = 0; i < 3; ++i) {
    pre += r0[i].re * r1[i].re + r0[i].im * r1[i].im;
    pim += r0[i].re * r1[i].im - r0[i].im * r1[i].re;
  }
  for (int i = 0; i < 3; ++i) {
    r1[i].re -= pre * r0[i].re - pim * r0[i].im;
    r1[i].im -= pre * r0[i].im + pim * r0[i].re;
  }
  double n1 = 0;
  for (int i = 0; i < 3; ++i) n1 += r1[i].re * r1[i].re + r1[i].im * r1[i].im;
  n1 = 1.0 / sqrt(n1);
  for (int i = 0; i < 3; ++i) { r1[i].re *= n1; r1[i].im *= n1; }
  for (int i = 0; i < 3; ++i) {
    int j = (i + 1) % 3, k = (i + 2) % 3;
    double cre = r0[j].re * r1[k].re - r0[j].im * r1[k].im - (r0[k].re * r1[j].re - r0[k].im * r1[j].im);
    double cim = r0[j].re * r1[k].im + r0[j].im * r1[k].re - (r0[k].re * r1[j].im + r0[k].im * r1[j].re);
    e[6 + i].re = cre;
    e[6 + i].im = -cim;
  }
  memcpy(u, e, sizeof(e));
}

/* Random SU(3) element for (seed, tag, index, sub): M_ij = sigma (g + i g'),
 * X = (M - M^dag)/2 minus its trace part, U = exp(X). */
static void random_su3(uint64_t seed, uint32_t tag, uint64_t index, uint32_t sub, double sigma, cplx *u) {
  cplx m[9], x[9];
  for (int j = 0; j < 9; ++j) {
    double g0, g1;
    gauss2(seed, tag, index, sub * 16u + (uint32_t)j, &g0, &g1);
    m[j].re = sigma * g0;
    m[j].im = sigma * g1;
  }
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      x[3 * i + j].re = 0.5 * (m[3 * i + j].re - m[3 * j + i].re);
      x[3 * i + j].im = 0.5 * (m[3 * i + j].im + m[3 * j + i].im);
    }
  double tr = (x[0].im + x[4].im + x[8].im) / 3.0;
  x[0].im -= tr; x[4].im -= tr; x[8].im -= tr;
  su3_exp(x, u);
}

/* ---- public entry points ------------------------------------------------ */

/* U[mu][site][3][3] complex for sites idx[0..n-1] (idx == NULL: sites 0..n-1).
 * Output is packed in the order of the list: out[mu][k][3][3]. */
void sg_gauge_su3(uint64_t seed, double sigma, const int64_t *idx, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    uint64_t s = idx ? (uint64_t)idx[k] : (uint64_t)k;
    for (int mu = 0; mu < 4; ++mu)
      random_su3(seed, SG_TAG_SU3, s, (uint32_t)mu, sigma, (cplx *)(out + 18 * (mu * n + k)));
  }
}

/* A[mu][site] ~ N(0, sigma^2). */
void sg_gauge_u1(uint64_t seed, double sigma, const int64_t *idx, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    uint64_t s = idx ? (uint64_t)idx[k] : (uint64_t)k;
    for (int mu = 0; mu < 4; ++mu) {
      double g0, g1;
      gauss2(seed, SG_TAG_U1, s, (uint32_t)mu, &g0, &g1);
      out[mu * n + k] = sigma * g0;
    }
  }
}

/* psi[site][4 spin][3 colour] complex, Re, Im ~ N(0, 1/2). */
void sg_spinor(uint64_t seed, const int64_t *idx, int64_t n, double *out) {
  const double h = 0.70710678118654752440084436210485;
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    uint64_t s = idx ? (uint64_t)idx[k] : (uint64_t)k;
    for (int c = 0; c < 12; ++c) {
      double g0, g1;
      gauss2(seed, SG_TAG_SPINOR, s, (uint32_t)c, &g0, &g1);
      out[24 * k + 2 * c] = h * g0;
      out[24 * k + 2 * c + 1] = h * g1;
    }
  }
}

/* Random SU(3) gauge-transformation field Omega[site][3][3]. */
void sg_transform_su3(uint64_t seed, double sigma, const int64_t *idx, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    uint64_t s = idx ? (uint64_t)idx[k] : (uint64_t)k;
    random_su3(seed, SG_TAG_TRANSFORM, s, 0u, sigma, (cplx *)(out + 18 * k));
  }
}

/* Generic real Gaussians: out[k] = sigma * N(0,1), counter (seed, tag, k). */
void sg_gaussian(uint64_t seed, uint32_t tag, double sigma, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    double g0, g1;
    gauss2(seed, SG_TAG_REAL + 16u * tag, (uint64_t)k, 0u, &g0, &g1);
    out[k] = sigma * g0;
  }
}

/* Real angles alpha[site] ~ N(0, sigma^2) for U(1) gauge transformations. */
void sg_angle(uint64_t seed, double sigma, const int64_t *idx, int64_t n, double *out) {
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n; ++k) {
    uint64_t s = idx ? (uint64_t)idx[k] : (uint64_t)k;
    double g0, g1;
    gauss2(seed, SG_TAG_ANGLE, s, 0u, &g0, &g1);
    out[k] = sigma * g0;
  }
}
