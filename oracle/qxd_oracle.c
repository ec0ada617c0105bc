/*
 * qxd oracle: a plain, slow FP64 CPU implementation of the Wilson-clover
 * operator with SU(3) x U(1) links under C* boundary conditions (openQ*D,
 * arXiv:1908.11673), its even-odd Schur complement, a CG solve, and the
 * convolution layers of the learned preconditioner.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the GPU path: it has its own geometry, its own gamma matrices, and evaluates
 * every formula as the paper writes it, with no spin projection, no chiral
 * block structure and no fusion.
 *
 * Conventions where the paper defers to other documents (written out once here
 * and, independently, in the GPU path):
 *   - chiral gamma basis, 2x2 blocks: g0 = [[0,-1],[-1,0]], gk = [[0,-i s_k],[i s_k,0]];
 *   - sigma_{mu nu} = (i/2)[g_mu, g_nu];
 *   - F_{mu nu} = (1/8)(Q_{mu nu} - Q_{nu mu}) from the four clover leaves
 *     (Luscher, Sint, Sommer, Weisz 1996), no trace removed;
 *   - site index x3 + L3 (x2 + L2 (x1 + L1ext x0)) on the extended lattice;
 *     parity (x0+x1+x2+x3) mod 2;
 *   - fermion field periodic in time unless t_antiperiodic is set.
 *
 * Fields: spinors are [site][spin 4][colour 3] complex; links U[mu][site][3][3]
 * (row, column); U(1) angles A[mu][site].  All on the extended lattice.
 *
 * Built with -O2 -ffp-contract=off so that no FMA contraction happens.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

typedef struct {
  int L[4];      /* physical extents */
  int Le[4];     /* extended extents (Le[1] = 2 L[1] when cstar >= 1) */
  int cstar;     /* number of C* directions, switched on in 1, 2, 3 order */
  int tanti;     /* fermion antiperiodic in time */
  int64_t V;     /* extended volume */
  int64_t *nb;   /* [V][4][2] neighbour sites (dir 0: +mu, 1: -mu) */
  double *nbs;   /* [V][4][2] fermion boundary sign of that hop */
  cplx *U;       /* [4][V][9] extended SU(3) links */
  double *A;     /* [4][V] extended U(1) angles */
  /* flavour */
  int qhat;
  double invqel, kappa, csw, cu1, m0;
  cplx *Vl;      /* [4][V][9] combined links U z^qhat */
  cplx *sw;      /* optional cache [V][12][12] of the SW term */
  cplx *blk;     /* optional cache [V][12][12] of the site blocks D(x,x) */
  cplx gam[4][4][4];
  cplx g5[4][4];
  cplx sig[4][4][4][4];
} or_ctx;

/* ------------------------------------------------------------------------
 * Geometry (Sec. 2.1: the extended lattice L0 x 2L1 x L2 x L3, periodic in
 * direction 1 with period 2L1; for the further C* directions k <= cstar,
 * stepping across the k boundary also shifts x1 by L1 (shifted boundary
 * conditions of the extended lattice); other directions periodic).
 * ---------------------------------------------------------------------- */

static int64_t site_of(const or_ctx *c, const int x[4]) {
  return (int64_t)x[3] + (int64_t)c->Le[3] * ((int64_t)x[2] + (int64_t)c->Le[2] * ((int64_t)x[1] + (int64_t)c->Le[1] * x[0]));
}

static void coords_of(const or_ctx *c, int64_t s, int x[4]) {
  x[3] = (int)(s % c->Le[3]); s /= c->Le[3];
  x[2] = (int)(s % c->Le[2]); s /= c->Le[2];
  x[1] = (int)(s % c->Le[1]); s /= c->Le[1];
  x[0] = (int)s;
}

/* One unit step from x along mu by dir = +1 or -1.  Returns the fermion sign. */
static double unit_step(const or_ctx *c, int x[4], int mu, int dir) {
  double sign = 1.0;
  x[mu] += dir;
  if (x[mu] < 0 || x[mu] >= c->Le[mu]) {
    x[mu] = (x[mu] + c->Le[mu]) % c->Le[mu];
    if (mu == 0 && c->tanti) sign = -1.0;
    if (mu >= 2 && mu <= c->cstar) x[1] = (x[1] + c->L[1]) % c->Le[1];
  }
  return sign;
}

or_ctx *or_create(int L0, int L1, int L2, int L3, int cstar, int tanti) {
  if (L0 < 2 || L1 < 2 || L2 < 2 || L3 < 2 || (L0 | L1 | L2 | L3) & 1 || cstar < 0 || cstar > 3) return NULL;
  or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
  c->L[0] = L0; c->L[1] = L1; c->L[2] = L2; c->L[3] = L3;
  for (int m = 0; m < 4; ++m) c->Le[m] = c->L[m];
  if (cstar >= 1) c->Le[1] = 2 * L1;
  c->cstar = cstar;
  c->tanti = tanti;
  c->V = (int64_t)c->Le[0] * c->Le[1] * c->Le[2] * c->Le[3];
  c->nb = (int64_t *)malloc(sizeof(int64_t) * 8 * c->V);
  c->nbs = (double *)malloc(sizeof(double) * 8 * c->V);
#pragma omp parallel for
  for (int64_t s = 0; s < c->V; ++s) {
    for (int mu = 0; mu < 4; ++mu)
      for (int d = 0; d < 2; ++d) {
        int x[4];
        coords_of(c, s, x);
        double sg = unit_step(c, x, mu, d == 0 ? +1 : -1);
        c->nb[8 * s + 2 * mu + d] = site_of(c, x);
        c->nbs[8 * s + 2 * mu + d] = sg;
      }
  }
  /* gamma matrices in the chiral basis */
  cplx pauli[3][2][2] = {{{0, 1}, {1, 0}}, {{0, -I}, {I, 0}}, {{1, 0}, {0, -1}}};
  memset(c->gam, 0, sizeof(c->gam));
  for (int a = 0; a < 2; ++a) {
    c->gam[0][a][2 + a] = -1;
    c->gam[0][2 + a][a] = -1;
  }
  for (int k = 1; k < 4; ++k)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        c->gam[k][a][2 + b] = -I * pauli[k - 1][a][b];
        c->gam[k][2 + a][b] = I * pauli[k - 1][a][b];
      }
  /* gamma5 = g0 g1 g2 g3 and sigma_{mu nu} = (i/2)[g_mu, g_nu] */
  cplx t1[4][4], t2[4][4];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += c->gam[0][i][k] * c->gam[1][k][j];
      t1[i][j] = s;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += t1[i][k] * c->gam[2][k][j];
      t2[i][j] = s;
    }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cplx s = 0;
      for (int k = 0; k < 4; ++k) s += t2[i][k] * c->gam[3][k][j];
      c->g5[i][j] = s;
    }
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu)
      for (int i = 0; i < 4; ++i)
        for (int j = 0; j < 4; ++j) {
          cplx s = 0;
          for (int k = 0; k < 4; ++k) s += c->gam[mu][i][k] * c->gam[nu][k][j] - c->gam[nu][i][k] * c->gam[mu][k][j];
          c->sig[mu][nu][i][j] = 0.5 * I * s;
        }
  return c;
}

void or_destroy(or_ctx *c) {
  if (!c) return;
  free(c->nb); free(c->nbs); free(c->U); free(c->A); free(c->Vl); free(c->sw); free(c->blk);
  free(c);
}

int64_t or_volume(const or_ctx *c) { return c->V; }

void or_extents(const or_ctx *c, int *Le) { for (int m = 0; m < 4; ++m) Le[m] = c->Le[m]; }

void or_neighbours(const or_ctx *c, int64_t *out, double *sign) {
  memcpy(out, c->nb, sizeof(int64_t) * 8 * c->V);
  if (sign) memcpy(sign, c->nbs, sizeof(double) * 8 * c->V);
}

/* x + d with d in {-1,0,1}^4: unit steps in direction order 0..3 (no sign). */
int64_t or_shift(const or_ctx *c, int64_t s, const int d[4]) {
  int x[4];
  coords_of(c, s, x);
  for (int mu = 0; mu < 4; ++mu)
    if (d[mu] != 0) unit_step(c, x, mu, d[mu]);
  return site_of(c, x);
}

/* parity of every extended site */
void or_parity(const or_ctx *c, int8_t *par) {
  for (int64_t s = 0; s < c->V; ++s) {
    int x[4];
    coords_of(c, s, x);
    par[s] = (int8_t)((x[0] + x[1] + x[2] + x[3]) & 1);
  }
}

/* ------------------------------------------------------------------------
 * Gauge fields on the extended lattice (Sec. 2.1, C* boundary conditions of
 * the gauge field: the mirror copy x + L1 e1 holds U* and -A).
 * ---------------------------------------------------------------------- */

static void alloc_gauge(or_ctx *c) {
  if (!c->U) c->U = (cplx *)malloc(sizeof(cplx) * 36 * c->V);
  if (!c->A) c->A = (double *)malloc(sizeof(double) * 4 * c->V);
}

/* U_phys[mu][s_phys][3][3], A_phys[mu][s_phys], s_phys = x3 + L3(x2 + L2(x1 + L1 x0)) */
void or_set_gauge_physical(or_ctx *c, const cplx *Up, const double *Ap) {
  alloc_gauge(c);
  int64_t Vp = (int64_t)c->L[0] * c->L[1] * c->L[2] * c->L[3];
#pragma omp parallel for
  for (int64_t s = 0; s < c->V; ++s) {
    int x[4];
    coords_of(c, s, x);
    int mirror = x[1] >= c->L[1];
    int x1 = mirror ? x[1] - c->L[1] : x[1];
    int64_t sp = (int64_t)x[3] + (int64_t)c->L[3] * ((int64_t)x[2] + (int64_t)c->L[2] * ((int64_t)x1 + (int64_t)c->L[1] * x[0]));
    for (int mu = 0; mu < 4; ++mu) {
      for (int k = 0; k < 9; ++k) {
        cplx u = Up[9 * (mu * Vp + sp) + k];
        c->U[9 * (mu * c->V + s) + k] = mirror ? conj(u) : u;
      }
      double a = Ap[mu * Vp + sp];
      c->A[mu * c->V + s] = mirror ? -a : a;
    }
  }
}

void or_set_gauge_extended(or_ctx *c, const cplx *Ue, const double *Ae) {
  alloc_gauge(c);
  memcpy(c->U, Ue, sizeof(cplx) * 36 * c->V);
  memcpy(c->A, Ae, sizeof(double) * 4 * c->V);
}

void or_get_gauge_extended(const or_ctx *c, cplx *Ue, double *Ae) {
  memcpy(Ue, c->U, sizeof(cplx) * 36 * c->V);
  memcpy(Ae, c->A, sizeof(double) * 4 * c->V);
}

/* ---- 3x3 helpers ------------------------------------------------------- */

static void m3_mul(const cplx *a, const cplx *b, cplx *r) {
  cplx t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cplx s = 0;
      for (int k = 0; k < 3; ++k) s += a[3 * i + k] * b[3 * k + j];
      t[3 * i + j] = s;
    }
  memcpy(r, t, sizeof(t));
}

static void m3_dag(const cplx *a, cplx *r) {
  cplx t[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t[3 * i + j] = conj(a[3 * j + i]);
  memcpy(r, t, sizeof(t));
}

static const cplx *link_U(const or_ctx *c, int64_t s, int mu) { return c->U + 9 * (mu * c->V + s); }
static double link_A(const or_ctx *c, int64_t s, int mu) { return c->A[mu * c->V + s]; }
static int64_t nbr(const or_ctx *c, int64_t s, int mu, int dir) { return c->nb[8 * s + 2 * mu + (dir > 0 ? 0 : 1)]; }
static double nbr_sign(const or_ctx *c, int64_t s, int mu, int dir) { return c->nbs[8 * s + 2 * mu + (dir > 0 ? 0 : 1)]; }

/* ------------------------------------------------------------------------
 * SW term (Sec. 2.3): csw_SU3 sum_{mu,nu} (i/4) sigma F + q csw_U1 sum (i/4) sigma A,
 * F from the four SU(3) clover leaves, A = (i / (4 q_el)) Im(sum of the four
 * U(1) plaquettes z_{mu nu} at x, x-mu, x-nu, x-mu-nu), q = qhat q_el.
 * ---------------------------------------------------------------------- */

/* Q_{mu nu}(x): sum of the four leaves, each a closed path from x, turning
 * from +mu towards +nu. */
static void clover_leaves(const or_ctx *c, int64_t x, int mu, int nu, cplx *Q) {
  cplx t[9], d[9];
  int64_t xpm = nbr(c, x, mu, +1), xpn = nbr(c, x, nu, +1);
  int64_t xmm = nbr(c, x, mu, -1), xmn = nbr(c, x, nu, -1);
  int64_t xmm_pn = nbr(c, xmm, nu, +1);  /* x - mu + nu */
  int64_t xmm_mn = nbr(c, xmm, nu, -1);  /* x - mu - nu */
  int64_t xmn_pm = nbr(c, xmn, mu, +1);  /* x - nu + mu */
  for (int k = 0; k < 9; ++k) Q[k] = 0;
  /* U(x,mu) U(x+mu,nu) U(x+nu,mu)^+ U(x,nu)^+ */
  m3_mul(link_U(c, x, mu), link_U(c, xpm, nu), t);
  m3_dag(link_U(c, xpn, mu), d); m3_mul(t, d, t);
  m3_dag(link_U(c, x, nu), d); m3_mul(t, d, t);
  for (int k = 0; k < 9; ++k) Q[k] += t[k];
  /* U(x,nu) U(x-mu+nu,mu)^+ U(x-mu,nu)^+ U(x-mu,mu) */
  m3_dag(link_U(c, xmm_pn, mu), d); m3_mul(link_U(c, x, nu), d, t);
  m3_dag(link_U(c, xmm, nu), d); m3_mul(t, d, t);
  m3_mul(t, link_U(c, xmm, mu), t);
  for (int k = 0; k < 9; ++k) Q[k] += t[k];
  /* U(x-mu,mu)^+ U(x-mu-nu,nu)^+ U(x-mu-nu,mu) U(x-nu,nu) */
  m3_dag(link_U(c, xmm, mu), t);
  m3_dag(link_U(c, xmm_mn, nu), d); m3_mul(t, d, t);
  m3_mul(t, link_U(c, xmm_mn, mu), t);
  m3_mul(t, link_U(c, xmn, nu), t);
  for (int k = 0; k < 9; ++k) Q[k] += t[k];
  /* U(x-nu,nu)^+ U(x-nu,mu) U(x-nu+mu,nu) U(x,mu)^+ */
  m3_dag(link_U(c, xmn, nu), t);
  m3_mul(t, link_U(c, xmn, mu), t);
  m3_mul(t, link_U(c, xmn_pm, nu), t);
  m3_dag(link_U(c, x, mu), d); m3_mul(t, d, t);
  for (int k = 0; k < 9; ++k) Q[k] += t[k];
}

/* U(1) plaquette z_{mu nu}(y) = z(y,mu) z(y+mu,nu) z(y+nu,mu)^* z(y,nu)^*  (unit charge) */
static cplx u1_plaq(const or_ctx *c, int64_t y, int mu, int nu) {
  cplx z1 = cexp(I * link_A(c, y, mu));
  cplx z2 = cexp(I * link_A(c, nbr(c, y, mu, +1), nu));
  cplx z3 = cexp(I * link_A(c, nbr(c, y, nu, +1), mu));
  cplx z4 = cexp(I * link_A(c, y, nu));
  return z1 * z2 * conj(z3) * conj(z4);
}

/* The field tensors at x: F[mu][nu] (3x3) and Ahat[mu][nu] (a scalar). */
void or_field_tensors(const or_ctx *c, int64_t x, cplx *F /*[4][4][9]*/, cplx *Ahat /*[4][4]*/) {
  double qel = 1.0 / c->invqel;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) {
      cplx *f = F + 9 * (4 * mu + nu);
      if (mu == nu) {
        for (int k = 0; k < 9; ++k) f[k] = 0;
        Ahat[4 * mu + nu] = 0;
        continue;
      }
      cplx Qa[9], Qb[9];
      clover_leaves(c, x, mu, nu, Qa);
      clover_leaves(c, x, nu, mu, Qb);
      for (int k = 0; k < 9; ++k) f[k] = 0.125 * (Qa[k] - Qb[k]);
      int64_t xm = nbr(c, x, mu, -1), xn = nbr(c, x, nu, -1);
      int64_t xmn = nbr(c, xm, nu, -1);
      cplx zs = u1_plaq(c, x, mu, nu) + u1_plaq(c, xm, mu, nu) + u1_plaq(c, xn, mu, nu) + u1_plaq(c, xmn, mu, nu);
      Ahat[4 * mu + nu] = I / (4.0 * qel) * cimag(zs);
    }
}

/* SW term at x as a 12x12 matrix indexed (3 spin + colour). */
static void sw_site(const or_ctx *c, int64_t x, cplx *sw) {
  cplx F[144], Ah[16];
  double q = (double)c->qhat / c->invqel;  /* physical charge q = qhat q_el */
  or_field_tensors(c, x, F, Ah);
  for (int k = 0; k < 144; ++k) sw[k] = 0;
  for (int mu = 0; mu < 4; ++mu)
    for (int nu = 0; nu < 4; ++nu) {
      if (mu == nu) continue;
      cplx E[9];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          E[3 * a + b] = c->csw * F[9 * (4 * mu + nu) + 3 * a + b] + (a == b ? q * c->cu1 * Ah[4 * mu + nu] : 0.0);
      for (int s = 0; s < 4; ++s)
        for (int t = 0; t < 4; ++t) {
          cplx sg = 0.25 * I * c->sig[mu][nu][s][t];
          if (sg == 0) continue;
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) sw[12 * (3 * s + a) + 3 * t + b] += sg * E[3 * a + b];
        }
    }
}

void or_sw_site(const or_ctx *c, int64_t x, cplx *sw) { sw_site(c, x, sw); }

/* Flavour: combined links V = U z^qhat (Sec. 2.3, covariant derivatives) and,
 * optionally, a cache of the SW term on every site. */
void or_set_flavour(or_ctx *c, int qhat, double invqel, double kappa, double csw, double cu1, int cache_sw) {
  c->qhat = qhat; c->invqel = invqel; c->kappa = kappa; c->csw = csw; c->cu1 = cu1;
  c->m0 = 1.0 / (2.0 * kappa) - 4.0;
  if (!c->Vl) c->Vl = (cplx *)malloc(sizeof(cplx) * 36 * c->V);
#pragma omp parallel for
  for (int64_t s = 0; s < c->V; ++s)
    for (int mu = 0; mu < 4; ++mu) {
      cplx zq = cexp(I * (double)qhat * link_A(c, s, mu));
      for (int k = 0; k < 9; ++k) c->Vl[9 * (mu * c->V + s) + k] = link_U(c, s, mu)[k] * zq;
    }
  free(c->sw);
  c->sw = NULL;
  free(c->blk);
  c->blk = NULL;
  if (cache_sw) {
    c->sw = (cplx *)malloc(sizeof(cplx) * 144 * c->V);
#pragma omp parallel for
    for (int64_t s = 0; s < c->V; ++s) sw_site(c, s, c->sw + 144 * s);
  }
}

void or_site_block(const or_ctx *c, int64_t x, cplx *M);

/* Cache the site blocks D(x,x) (read off by probing) on every site. */
void or_cache_blocks(or_ctx *c) {
  free(c->blk);
  c->blk = NULL;
  cplx *b = (cplx *)malloc(sizeof(cplx) * 144 * c->V);
#pragma omp parallel for
  for (int64_t s = 0; s < c->V; ++s) or_site_block(c, s, b + 144 * s);
  c->blk = b;
}

/* ------------------------------------------------------------------------
 * The Dirac operator (Sec. 2.3):  D = m0 + Dw + dD_sw, with
 *   Dw = sum_mu (1/2) { g_mu (nabla_mu + nabla*_mu) - nabla*_mu nabla_mu },
 *   nabla_mu psi(x)  = V(x,mu) psi(x+mu) - psi(x),
 *   nabla*_mu psi(x) = psi(x) - V(x-mu,mu)^+ psi(x-mu),
 *   V = U z^qhat,  a m0 = 1/(2 kappa) - 4.
 * Evaluated at one site from a field accessor, so the same code serves the
 * full operator, sampled sites, and probing of site blocks.
 * ---------------------------------------------------------------------- */

typedef struct {
  void (*get)(const void *ctx, int64_t site, cplx *out12);
  const void *ctx;
} field;

static void get_dense(const void *ctx, int64_t s, cplx *o) { memcpy(o, (const cplx *)ctx + 12 * s, sizeof(cplx) * 12); }

static const cplx *Vlink(const or_ctx *c, int64_t s, int mu) { return c->Vl + 9 * (mu * c->V + s); }

/* colour matrix on each spin component: out = M psi or M^+ psi */
static void col_mul(const cplx *M, const cplx *psi, cplx *out, int dag) {
  for (int s = 0; s < 4; ++s)
    for (int a = 0; a < 3; ++a) {
      cplx acc = 0;
      for (int b = 0; b < 3; ++b) acc += (dag ? conj(M[3 * b + a]) : M[3 * a + b]) * psi[3 * s + b];
      out[3 * s + a] = acc;
    }
}

static void spin_mul(const cplx g[4][4], const cplx *psi, cplx *out) {
  for (int s = 0; s < 4; ++s)
    for (int a = 0; a < 3; ++a) {
      cplx acc = 0;
      for (int t = 0; t < 4; ++t) acc += g[s][t] * psi[3 * t + a];
      out[3 * s + a] = acc;
    }
}

static void dirac_site(const or_ctx *c, const field *f, int64_t x, cplx *out) {
  cplx px[12], pp[12], pm[12], fwd[12], bwd[12], nm[12], lap[12], t[12], g[12];
  f->get(f->ctx, x, px);
  for (int i = 0; i < 12; ++i) out[i] = c->m0 * px[i];
  for (int mu = 0; mu < 4; ++mu) {
    int64_t xp = nbr(c, x, mu, +1), xm = nbr(c, x, mu, -1);
    double sp = nbr_sign(c, x, mu, +1), sm = nbr_sign(c, x, mu, -1);
    f->get(f->ctx, xp, pp);
    f->get(f->ctx, xm, pm);
    for (int i = 0; i < 12; ++i) { pp[i] *= sp; pm[i] *= sm; }
    /* (nabla psi)(x) */
    col_mul(Vlink(c, x, mu), pp, t, 0);
    for (int i = 0; i < 12; ++i) fwd[i] = t[i] - px[i];
    /* (nabla* psi)(x) */
    col_mul(Vlink(c, xm, mu), pm, t, 1);
    for (int i = 0; i < 12; ++i) bwd[i] = px[i] - t[i];
    /* (nabla psi)(x - mu) = V(x-mu,mu) psi(x) - psi(x-mu) */
    col_mul(Vlink(c, xm, mu), px, t, 0);
    for (int i = 0; i < 12; ++i) nm[i] = t[i] - pm[i];
    /* (nabla* nabla psi)(x) = (nabla psi)(x) - V(x-mu,mu)^+ (nabla psi)(x-mu) */
    col_mul(Vlink(c, xm, mu), nm, t, 1);
    for (int i = 0; i < 12; ++i) lap[i] = fwd[i] - t[i];
    for (int i = 0; i < 12; ++i) t[i] = fwd[i] + bwd[i];
    spin_mul(c->gam[mu], t, g);
    for (int i = 0; i < 12; ++i) out[i] += 0.5 * (g[i] - lap[i]);
  }
  cplx swl[144];
  const cplx *sw = c->sw ? c->sw + 144 * x : swl;
  if (!c->sw) sw_site(c, x, swl);
  for (int i = 0; i < 12; ++i) {
    cplx acc = 0;
    for (int j = 0; j < 12; ++j) acc += sw[12 * i + j] * px[j];
    out[i] += acc;
  }
}

/* full operator on the extended lattice */
void or_dirac(const or_ctx *c, const cplx *psi, cplx *out) {
  field f = {get_dense, psi};
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < c->V; ++s) dirac_site(c, &f, s, out + 12 * s);
}

/* (D psi)(x) on a list of sites */
void or_dirac_sites(const or_ctx *c, const cplx *psi, const int64_t *sites, int64_t n, cplx *out) {
  field f = {get_dense, psi};
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t k = 0; k < n; ++k) dirac_site(c, &f, sites[k], out + 12 * k);
}

/* ------------------------------------------------------------------------
 * Even-odd decomposition (Sec. 2.3): D_hat = D_ee - D_eo D_oo^{-1} D_oe.
 * D_oo is site-diagonal; its 12x12 block at x is read off D by probing with
 * unit vectors supported on x.
 * ---------------------------------------------------------------------- */

typedef struct { int64_t site; int comp; } probe_ctx;

static void get_probe(const void *ctx, int64_t s, cplx *o) {
  const probe_ctx *p = (const probe_ctx *)ctx;
  for (int i = 0; i < 12; ++i) o[i] = 0;
  if (s == p->site) o[p->comp] = 1.0;
}

/* 12x12 block D(x,x), row-major: M[12 i + j] = (D e_{x,j})_i(x) */
void or_site_block(const or_ctx *c, int64_t x, cplx *M) {
  for (int j = 0; j < 12; ++j) {
    probe_ctx p = {x, j};
    field f = {get_probe, &p};
    cplx col[12];
    dirac_site(c, &f, x, col);
    for (int i = 0; i < 12; ++i) M[12 * i + j] = col[i];
  }
}

/* Solve M y = b (12x12) by Gaussian elimination with partial pivoting.
 * Returns the smallest pivot magnitude. */
static double solve12(const cplx *Min, const cplx *b, cplx *y) {
  cplx M[144], r[12];
  memcpy(M, Min, sizeof(M));
  memcpy(r, b, sizeof(r));
  double minpiv = INFINITY;
  for (int k = 0; k < 12; ++k) {
    int p = k;
    for (int i = k + 1; i < 12; ++i)
      if (cabs(M[12 * i + k]) > cabs(M[12 * p + k])) p = i;
    if (p != k) {
      for (int j = 0; j < 12; ++j) { cplx t = M[12 * k + j]; M[12 * k + j] = M[12 * p + j]; M[12 * p + j] = t; }
      cplx t = r[k]; r[k] = r[p]; r[p] = t;
    }
    double a = cabs(M[12 * k + k]);
    if (a < minpiv) minpiv = a;
    for (int i = k + 1; i < 12; ++i) {
      cplx l = M[12 * i + k] / M[12 * k + k];
      for (int j = k; j < 12; ++j) M[12 * i + j] -= l * M[12 * k + j];
      r[i] -= l * r[k];
    }
  }
  for (int k = 11; k >= 0; --k) {
    cplx s = r[k];
    for (int j = k + 1; j < 12; ++j) s -= M[12 * k + j] * y[j];
    y[k] = s / M[12 * k + k];
  }
  return minpiv;
}

static int parity_of(const or_ctx *c, int64_t s) {
  int x[4];
  coords_of(c, s, x);
  return (x[0] + x[1] + x[2] + x[3]) & 1;
}

/* field equal to psi on sites of parity p and zero elsewhere */
typedef struct { const or_ctx *c; const cplx *psi; int p; } restrict_ctx;
static void get_restricted(const void *ctx, int64_t s, cplx *o) {
  const restrict_ctx *r = (const restrict_ctx *)ctx;
  if (parity_of(r->c, s) == r->p) memcpy(o, r->psi + 12 * s, sizeof(cplx) * 12);
  else for (int i = 0; i < 12; ++i) o[i] = 0;
}

/* D_oo^{-1} v at odd site y */
static void doo_inv(const or_ctx *c, int64_t y, const cplx *v, cplx *out) {
  cplx M[144];
  if (c->blk) memcpy(M, c->blk + 144 * y, sizeof(M));
  else or_site_block(c, y, M);
  solve12(M, v, out);
}

/* phi = psi_e on even sites, t_o = -D_oo^{-1} D_oe psi_e on odd sites, computed
 * on demand.  Then (D phi)_e = D_hat psi_e and (D phi)_o = 0. */
static void get_schur_phi(const void *ctx, int64_t s, cplx *o) {
  const restrict_ctx *r = (const restrict_ctx *)ctx;
  if (parity_of(r->c, s) == 0) { memcpy(o, r->psi + 12 * s, sizeof(cplx) * 12); return; }
  restrict_ctx e = {r->c, r->psi, 0};
  field fe = {get_restricted, &e};
  cplx w[12], t[12];
  dirac_site(r->c, &fe, s, w);  /* (D_oe psi_e)(s) */
  doo_inv(r->c, s, w, t);
  for (int i = 0; i < 12; ++i) o[i] = -t[i];
}

static void g5_apply(const or_ctx *c, const cplx *in, cplx *out) { spin_mul(c->g5, in, out); }

/* D_hat psi_e on the listed even sites; dagger: gamma5 D_hat gamma5.
 * psi is a full-lattice field of which only the even sites are read. */
void or_schur_sites(const or_ctx *c, const cplx *psi, const int64_t *sites, int64_t n, cplx *out, int dagger) {
  cplx *src = (cplx *)psi;
  if (dagger) {
    src = (cplx *)malloc(sizeof(cplx) * 12 * c->V);
#pragma omp parallel for
    for (int64_t s = 0; s < c->V; ++s) g5_apply(c, psi + 12 * s, src + 12 * s);
  }
  restrict_ctx r = {c, src, 0};
  field f = {get_schur_phi, &r};
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t k = 0; k < n; ++k) {
    cplx o[12];
    dirac_site(c, &f, sites[k], o);
    if (dagger) g5_apply(c, o, out + 12 * k);
    else memcpy(out + 12 * k, o, sizeof(o));
  }
  if (dagger) free(src);
}

/* D_hat on the whole even sub-lattice (odd sites of out set to zero).
 * Two literal passes: t_o = -D_oo^{-1} (D psi_e)_o, then out_e = (D (psi_e + t_o))_e. */
void or_schur(const or_ctx *c, const cplx *psi, cplx *out, int dagger) {
  int64_t V = c->V;
  cplx *src = (cplx *)malloc(sizeof(cplx) * 12 * V);
  cplx *phi = (cplx *)malloc(sizeof(cplx) * 12 * V);
#pragma omp parallel for
  for (int64_t s = 0; s < V; ++s) {
    if (dagger) g5_apply(c, psi + 12 * s, src + 12 * s);
    else memcpy(src + 12 * s, psi + 12 * s, sizeof(cplx) * 12);
  }
  restrict_ctx e = {c, src, 0};
  field fe = {get_restricted, &e};
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < V; ++s) {
    if (parity_of(c, s) == 0) { memcpy(phi + 12 * s, src + 12 * s, sizeof(cplx) * 12); continue; }
    cplx w[12], t[12];
    dirac_site(c, &fe, s, w);
    doo_inv(c, s, w, t);
    for (int i = 0; i < 12; ++i) phi[12 * s + i] = -t[i];
  }
  field f = {get_dense, phi};
#pragma omp parallel for schedule(static)
  for (int64_t s = 0; s < V; ++s) {
    cplx o[12];
    if (parity_of(c, s) == 1) { for (int i = 0; i < 12; ++i) out[12 * s + i] = 0; continue; }
    dirac_site(c, &f, s, o);
    if (dagger) g5_apply(c, o, out + 12 * s);
    else memcpy(out + 12 * s, o, sizeof(o));
  }
  free(src);
  free(phi);
}

/* Smallest pivot magnitude of the site blocks D(x,x) over all sites. */
double or_min_block_pivot(const or_ctx *c) {
  double mn = INFINITY;
#pragma omp parallel for reduction(min : mn)
  for (int64_t s = 0; s < c->V; ++s) {
    cplx M[144], b[12] = {0}, y[12];
    or_site_block(c, s, M);
    double p = solve12(M, b, y);
    if (p < mn) mn = p;
  }
  return mn;
}

/* bhat_e = b_e - D_eo D_oo^{-1} b_o  (odd sites of out zero) */
void or_eo_source(const or_ctx *c, const cplx *b, cplx *out) {
  int64_t V = c->V;
  cplx *t = (cplx *)calloc((size_t)12 * V, sizeof(cplx));
#pragma omp parallel for
  for (int64_t s = 0; s < V; ++s)
    if (parity_of(c, s) == 1) doo_inv(c, s, b + 12 * s, t + 12 * s);
  field f = {get_dense, t};
#pragma omp parallel for
  for (int64_t s = 0; s < V; ++s) {
    if (parity_of(c, s) == 1) { for (int i = 0; i < 12; ++i) out[12 * s + i] = 0; continue; }
    cplx w[12];
    dirac_site(c, &f, s, w);  /* (D_eo t_o)(s): t vanishes on even sites */
    for (int i = 0; i < 12; ++i) out[12 * s + i] = b[12 * s + i] - w[i];
  }
  free(t);
}

/* x_o = D_oo^{-1} (b_o - D_oe x_e); x_e copied from xe. */
void or_eo_reconstruct(const or_ctx *c, const cplx *xe, const cplx *b, cplx *x) {
  int64_t V = c->V;
  restrict_ctx e = {c, xe, 0};
  field fe = {get_restricted, &e};
#pragma omp parallel for
  for (int64_t s = 0; s < V; ++s) {
    if (parity_of(c, s) == 0) { memcpy(x + 12 * s, xe + 12 * s, sizeof(cplx) * 12); continue; }
    cplx w[12], r[12];
    dirac_site(c, &fe, s, w);
    for (int i = 0; i < 12; ++i) r[i] = b[12 * s + i] - w[i];
    doo_inv(c, s, r, x + 12 * s);
  }
}

/* ------------------------------------------------------------------------
 * CG on the normal equations of the Schur system (Sec. 4.4 names CG among
 * the solvers): minimises |bhat - D_hat x| over the Krylov space of
 * D_hat^+ D_hat.  The residual r = bhat - D_hat x is carried along; at claimed
 * convergence it is recomputed from x and the iteration continues if the
 * recomputed value misses the target.  Vectors are full-lattice fields whose
 * odd sites are zero.  Returns iterations, or -1 without convergence.
 * ---------------------------------------------------------------------- */

static double dot_re(int64_t n, const cplx *a, const cplx *b) {
  double s = 0;
  for (int64_t i = 0; i < n; ++i) s += creal(conj(a[i]) * b[i]);
  return s;
}

int or_cg(const or_ctx *c, const cplx *bhat, cplx *x, double tol_abs, int nmx, double *res_out) {
  int64_t n = 12 * c->V;
  cplx *r = (cplx *)malloc(sizeof(cplx) * n), *z = (cplx *)malloc(sizeof(cplx) * n);
  cplx *p = (cplx *)malloc(sizeof(cplx) * n), *w = (cplx *)malloc(sizeof(cplx) * n);
  for (int64_t i = 0; i < n; ++i) x[i] = 0, r[i] = bhat[i];
  or_schur(c, r, z, 1);
  memcpy(p, z, sizeof(cplx) * n);
  double zz = dot_re(n, z, z), rr = dot_re(n, r, r);
  int it = 0, ok = 0;
  while (it < nmx) {
    if (sqrt(rr) <= tol_abs) {
      or_schur(c, x, w, 0);
      for (int64_t i = 0; i < n; ++i) r[i] = bhat[i] - w[i];
      rr = dot_re(n, r, r);
      if (sqrt(rr) <= tol_abs) { ok = 1; break; }
      or_schur(c, r, z, 1);
      memcpy(p, z, sizeof(cplx) * n);
      zz = dot_re(n, z, z);
    }
    or_schur(c, p, w, 0);
    double alpha = zz / dot_re(n, w, w);
    for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * w[i]; }
    or_schur(c, r, z, 1);
    double zz1 = dot_re(n, z, z);
    double beta = zz1 / zz;
    zz = zz1;
    for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
    rr = dot_re(n, r, r);
    ++it;
  }
  if (!ok) {
    or_schur(c, x, w, 0);
    for (int64_t i = 0; i < n; ++i) r[i] = bhat[i] - w[i];
    rr = dot_re(n, r, r);
    ok = sqrt(rr) <= tol_abs;
  }
  if (res_out) *res_out = sqrt(rr);
  free(r); free(z); free(p); free(w);
  return ok ? it : -1;
}

/* ------------------------------------------------------------------------
 * Learned preconditioner layers: a 3^4-tap convolution on the extended
 * lattice whose taps follow the C* neighbour map (x + d is a composition of
 * unit steps), its adjoint (a scatter, the literal transpose) and its weight
 * gradient.  W[tap][cout][cin], tap = 27(d0+1) + 9(d1+1) + 3(d2+1) + (d3+1);
 * activations [site][channel].
 * ---------------------------------------------------------------------- */

static void tap_offsets(int tap, int d[4]) {
  d[0] = tap / 27 - 1;
  d[1] = (tap / 9) % 3 - 1;
  d[2] = (tap / 3) % 3 - 1;
  d[3] = tap % 3 - 1;
}

void or_nn_conv(const or_ctx *c, int cin, int cout, const double *W, const double *h, double *y) {
#pragma omp parallel for schedule(static)
  for (int64_t x = 0; x < c->V; ++x) {
    double acc[64];
    for (int o = 0; o < cout; ++o) acc[o] = 0;
    for (int tap = 0; tap < 81; ++tap) {
      int d[4];
      tap_offsets(tap, d);
      int64_t xs = or_shift(c, x, d);
      for (int o = 0; o < cout; ++o)
        for (int i = 0; i < cin; ++i) acc[o] += W[((int64_t)tap * cout + o) * cin + i] * h[xs * cin + i];
    }
    for (int o = 0; o < cout; ++o) y[x * cout + o] = acc[o];
  }
}

/* dh = conv^T g : every output x sends W^T g(x) back to x + d (serial scatter) */
void or_nn_conv_adjoint(const or_ctx *c, int cin, int cout, const double *W, const double *g, double *dh) {
  memset(dh, 0, sizeof(double) * cin * c->V);
  for (int64_t x = 0; x < c->V; ++x)
    for (int tap = 0; tap < 81; ++tap) {
      int d[4];
      tap_offsets(tap, d);
      int64_t xs = or_shift(c, x, d);
      for (int i = 0; i < cin; ++i) {
        double s = 0;
        for (int o = 0; o < cout; ++o) s += W[((int64_t)tap * cout + o) * cin + i] * g[x * cout + o];
        dh[xs * cin + i] += s;
      }
    }
}

/* dW[tap][o][i] = sum_x g(x)[o] h(x + d)[i] */
void or_nn_conv_wgrad(const or_ctx *c, int cin, int cout, const double *g, const double *h, double *dW) {
#pragma omp parallel for schedule(static)
  for (int tap = 0; tap < 81; ++tap) {
    int d[4];
    tap_offsets(tap, d);
    for (int o = 0; o < cout; ++o)
      for (int i = 0; i < cin; ++i) dW[((int64_t)tap * cout + o) * cin + i] = 0;
    for (int64_t x = 0; x < c->V; ++x) {
      int64_t xs = or_shift(c, x, d);
      for (int o = 0; o < cout; ++o)
        for (int i = 0; i < cin; ++i) dW[((int64_t)tap * cout + o) * cin + i] += g[x * cout + o] * h[xs * cin + i];
    }
  }
}
