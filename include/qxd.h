/*
 * qxd.h -- C ABI of libqxd: the Wilson-clover operator with SU(3) x U(1)^qhat
 * links under C* boundary conditions on MI355X (gfx950), its even-odd Schur
 * complement, and the Krylov solves built on it (openQ*D, arXiv:1908.11673).
 *
 * Paper references are to sections and equations of arXiv:1908.11673:
 *   Sec. 2.1  C* boundary conditions, the extended (orbifold) lattice
 *   Sec. 2.3  the Dirac operator: D = m0 + Dw + dD_sw, the covariant
 *             derivatives with U z^qhat, the SU(3) and U(1) SW terms, and the
 *             even-odd preconditioned operator D_hat = D_ee - D_eo D_oo^-1 D_oe
 *   Sec. 4.4  the solvers (CG on D_hat^+ D_hat, GCR) and the residue 1e-10
 *
 * Conventions the paper leaves to other documents:
 *   - chiral gamma basis, 2x2 blocks: g0 = [[0,-1],[-1,0]], gk = [[0,-i s_k],[i s_k,0]],
 *     gamma5 = diag(1,1,-1,-1); sigma_{mu nu} = (i/2)[g_mu, g_nu];
 *   - F_{mu nu} = (1/8)(Q_{mu nu} - Q_{mu nu}^+) from the four clover leaves, no
 *     trace removed; the U(1) tensor is built from unit-charge plaquettes, so the
 *     SW term carries u1csw * qhat * (i/4) Im(sum of the four z_{mu nu}) and does
 *     not depend on invqel;
 *   - the diagonal of D is 1/(2 kappa) (a m0 = 1/(2 kappa) - 4);
 *   - fermions periodic in time unless t_antiperiodic is set.
 *
 * ---------------------------------------------------------------------------
 * Lattice and layouts
 *
 * Physical extents L0 (time), L1, L2, L3, all even and >= 2.  With cstar >= 1
 * the library works on the extended lattice L0 x 2L1 x L2 x L3 (Sec. 2.1):
 * direction 1 is periodic with period 2L1, and for 2 <= k <= cstar a hop across
 * the k boundary also moves x1 by L1.  Canonical site index on the extended
 * lattice: s = x3 + L3 (x2 + L2 (x1 + L1ext x0)); parity (x0+x1+x2+x3) mod 2;
 * the half index of a site within its parity is s / 2.  Ve = V / 2.
 *
 * Canonical (AoS) spinor: [V][4 spin][3 colour] complex128, interleaved re, im.
 * Device (SoA even-odd, "eo") spinor of precision p:
 *   half field (one parity):  F64  [12 components][Ve] complex128
 *                             F32  [6 pairs][Ve] (2 complex64 per 16 bytes)
 *                             BF16 [3 quads][Ve] (4 complex bf16 per 16 bytes)
 *   full field: the even half followed by the odd half.
 * Component c = 3 spin + colour.  Sizes in bytes: 192 Ve (F64), 96 Ve (F32),
 * 48 Ve (BF16) per half field.
 *
 * Every field pointer is a caller-owned device pointer unless stated.  All
 * calls are asynchronous on the given HIP stream (a hipStream_t passed as
 * void*, NULL for the null stream) except where stated; the solvers block
 * until their statistics are final.  One handle per host thread.
 *
 * Errors: every call returns a qxd_status; nothing throws or aborts across the
 * ABI.  On an error the outputs are unspecified and the handle stays usable.
 */
#ifndef QXD_H
#define QXD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QXD_OK = 0,
  QXD_EINVAL = 1,     /* bad argument (NULL pointer, size, enum value) */
  QXD_EGEOM = 2,      /* odd or too small extent, cstar outside 0..3, volume too large */
  QXD_ENOMEM = 3,     /* device allocation failed */
  QXD_ESINGULAR = 4,  /* a clover block has |pivot| < 1e-14 |H| */
  QXD_ENAN = 5,       /* a non-finite value reached a solver reduction */
  QXD_ENOCONV = 6,    /* the iteration limit was reached before the target */
  QXD_EHIP = 7,       /* a HIP runtime call failed */
  QXD_ESTATE = 8,     /* call out of order (e.g. apply before clover_invert) */
  QXD_ESCRATCH = 9,   /* the lattice needs more than the static workspace of a no-allocation call */
  QXD_EIO = 10        /* a file could not be written or read, or is not a valid network file */
} qxd_status;

typedef enum { QXD_F64 = 0, QXD_F32 = 1, QXD_BF16 = 2 } qxd_prec;

typedef struct {
  int L[4];            /* physical L0 (time), L1, L2, L3: even, >= 2 */
  int cstar;           /* C* directions 0..3, switched on in 1, 2, 3 order (Sec. 2.1) */
  int t_antiperiodic;  /* 1: fermion sign -1 on the time wrap */
} qxd_geom;

typedef struct {
  int qhat;            /* integer charge q / q_el (Sec. 2.3) */
  double invqel;       /* 1 / q_el; does not enter the operator (it cancels) */
  double kappa;        /* hopping parameter, diagonal 1/(2 kappa) */
  double su3csw;       /* SU(3) SW coefficient */
  double u1csw;        /* U(1) SW coefficient (1 at tree level) */
} qxd_flavour;

typedef struct {
  double min_pivot;    /* smallest |pivot| met in the 6x6 block inversions */
  double max_norm;     /* largest max-abs entry of a 6x6 block */
  int64_t n_singular;  /* blocks with |pivot| < 1e-14 max-abs entry */
} qxd_clover_stats;

typedef struct {
  int nmx;             /* iteration limit (CG: iterations; FGCR: inner steps in total) */
  double res;          /* target true relative residual |b - D x| / |b| (full lattice) */
  int inner_prec;      /* qxd_prec of the inner CG / FGCR operator (F64: no defect correction) */
  double inner_res;    /* relative residual reduction asked of each inner solve (0: 1e-5 for F32, 1e-3 for BF16) */
  int nkv;             /* FGCR restart length (1..24; 0: 16) */
  int max_outer;       /* defect-correction steps limit */
  int check_every;     /* CG: read the residual back every this many iterations */
  int fallback_after;  /* NN FGCR: inner steps without progress before dropping M */
  int sap_ncy;         /* FGCR: > 0 selects the SAP preconditioner with this many cycles (net must be NULL) */
  int sap_nmr;         /* SAP: minimal-residual steps per block solve */
  int sap_plain;       /* SAP: 0 (default) even-odd preconditioned block solves, 1 plain (see qxd_sap_apply) */
  int dfl_nc;          /* deflation: coarse GCR steps per preconditioner application (1..QXD_DFL_MAXNC; 0: 16) */
} qxd_solver_params;

typedef struct {
  int status;          /* qxd_status of the solve */
  int outer_it;        /* defect-correction steps */
  int inner_it;        /* CG iterations or FGCR steps, summed */
  int64_t schur_applies; /* D_hat or D_hat^+ applications, all precisions */
  int64_t nn_applies;  /* preconditioner network applications */
  double true_residual;/* FP64 |b - D x| / |b| on the full lattice, recomputed */
  double t_ms;         /* wall time of the call */
  int fell_back;       /* 1 if the preconditioner was dropped */
  int64_t sap_applies; /* SAP preconditioner applications */
} qxd_solver_stats;

typedef struct qxd_handle qxd_handle;
typedef struct qxd_nn qxd_nn;
typedef struct qxd_dfl qxd_dfl;

/* Status name for printing. */
const char *qxd_status_string(qxd_status s);

/* Create a handle for the geometry (Sec. 2.1).  Checks extents and cstar on
 * the host before any allocation: QXD_EGEOM on odd or < 2 extents, cstar
 * outside 0..3, or an extended volume >= 2^31.  Device: the current one. */
qxd_status qxd_create(const qxd_geom *g, qxd_handle **h);
qxd_status qxd_destroy(qxd_handle *h);

/* Extended volume V and Ve = V/2. */
qxd_status qxd_volume(const qxd_handle *h, int64_t *V, int64_t *Ve);

/* Release the memory a set-up handle no longer needs for applying D, D_hat or
 * solving: the device copy of the physical gauge field, every solver and Schur
 * workspace, and the FP32 / bf16 copies of the links and clover blocks (all
 * of these are made again when next used; the copies from the FP64 links and
 * blocks, which stay).  The handle makes a lower-precision copy only when a
 * call first needs it (an FP32 or bf16 apply or solve, SAP, deflation), so an
 * FP64-only computation never holds one.  Afterwards qxd_set_flavour and
 * qxd_clover_build return QXD_ESTATE until qxd_set_gauge is called again.  On
 * the largest lattices this is what leaves room for the solver vectors (at
 * 128 x 64^3 physical the FP64 operator alone is 97 GB).  Synchronises the
 * device. */
qxd_status qxd_trim(qxd_handle *h);

/* Gauge fields on the physical lattice: U_phys [4][Vphys][3][3] complex128 (row,
 * column), A_phys [4][Vphys] float64, Vphys = L0 L1 L2 L3, physical site index
 * x3 + L3 (x2 + L2 (x1 + L1 x0)).  on_device != 0: device pointers, else host
 * pointers (copied synchronously).  The library keeps its own copy and fills the
 * mirror half U(x + L1 e1) = U(x)*, A(x + L1 e1) = -A(x) itself (Sec. 2.1). */
qxd_status qxd_set_gauge(qxd_handle *h, const double *U_phys, const double *A_phys, int on_device, void *stream);

/* Select the flavour and build the combined links V(x,mu) = U(x,mu) z(x,mu)^qhat
 * (Sec. 2.3, covariant derivatives) on the extended lattice in FP64 (FP32 and
 * bf16 copies follow on first use).  Invalidates the clover until the next
 * clover_build/invert.
 * QXD_ESTATE without a gauge field (none set yet, or released by qxd_trim). */
qxd_status qxd_set_flavour(qxd_handle *h, const qxd_flavour *f, void *stream);

/* SW term (Sec. 2.3): the site-diagonal 1/(2 kappa) + dD_sw on every site, as two
 * Hermitian 6x6 chirality blocks.  QXD_ESTATE without a flavour or after
 * qxd_trim released the gauge field. */
qxd_status qxd_clover_build(qxd_handle *h, void *stream);

/* Invert the odd-site blocks (D_oo^-1 in Sec. 2.3's Schur complement) in FP64
 * by Gauss-Jordan elimination with partial pivoting (FP32 copies follow on
 * first use).
 * Synchronous (reads the statistics back); QXD_ESINGULAR if any block is
 * numerically singular. */
qxd_status qxd_clover_invert(qxd_handle *h, qxd_clover_stats *stats, void *stream);

/* out = D in on the full extended lattice (Sec. 2.3), eo layout of precision p,
 * full fields.  out and in must not overlap. */
qxd_status qxd_dw_apply(qxd_handle *h, qxd_prec p, void *out, const void *in, void *stream);

/* out_e = D_hat in_e (dagger = 0) or D_hat^+ in_e = gamma5 D_hat gamma5 in_e
 * (dagger = 1) (Sec. 2.3), even half fields of precision p.  Uses an internal
 * odd half field as workspace.  out_e and in_e must not overlap. */
qxd_status qxd_dw_eo_schur(qxd_handle *h, qxd_prec p, int dagger, void *out_e, const void *in_e, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * out_e = D_hat in_e / D_hat^+ in_e as qxd_dw_eo_schur, with the same kernels
 * and bit-identical results, but the odd half field of workspace is taken from
 * a static device array of QXD_NOALLOC_SCRATCH_BYTES per GPU (held from the
 * library's first use on a GPU until the process ends) instead of a handle
 * buffer allocated on first use; the call allocates and frees nothing.
 * QXD_ESCRATCH when the half field (192 Ve bytes F64, 96 Ve F32, 48 Ve BF16)
 * exceeds the array: up to Ve = 349,525 in F64, 699,050 in F32, 1,398,101 in
 * BF16.  QXD_EINVAL when the current device is not the handle's; QXD_ESTATE
 * before the clover inverse and, for F32 / BF16, while the handle holds no
 * current copy of the operator in that precision (made by the first F32 /
 * BF16 qxd_dw_eo_schur or solve, released by qxd_trim).  All calls on
 * one GPU share its array, which keeps the last call's contents: calls that
 * overlap in time on one GPU (several streams or host threads) race; serialise
 * them.  Nothing in the array needs to start at zero. */
#define QXD_NOALLOC_SCRATCH_BYTES (64u << 20)
qxd_status qxd_dw_eo_schur_noalloc(qxd_handle *h, qxd_prec p, int dagger, void *out_e, const void *in_e,
                                   void *stream);

/* bhat_e = b_e - D_eo D_oo^-1 b_o  (F64; b full field, bhat_e even half field). */
qxd_status qxd_eo_source(qxd_handle *h, void *bhat_e, const void *b, void *stream);

/* x = (x_e, D_oo^-1 (b_o - D_oe x_e))  (F64; x, b full fields, x_e even half). */
qxd_status qxd_eo_reconstruct(qxd_handle *h, void *x, const void *x_e, const void *b, void *stream);

/* Convert between the canonical AoS layout and the eo layout of precision p.
 * aos: device pointer to [V][4][3] complex128 (full lattice); soa: full field.
 * FP64 -> FP32 -> BF16 rounding is to nearest even. */
qxd_status qxd_pack(qxd_handle *h, qxd_prec p, void *soa, const double *aos, void *stream);
qxd_status qxd_unpack(qxd_handle *h, qxd_prec p, double *aos, const void *soa, void *stream);

/* Solve D x = b to |b - D x| / |b| <= params->res by CG on the normal equations
 * of the Schur system (Sec. 4.4): source preparation, CG, and reconstruction;
 * the residual is recomputed in FP64 on the full lattice before returning.
 * inner_prec F64: CG in FP64.  F32 or BF16: an FP64 defect-correction loop
 * (r = bhat - D_hat x in FP64, x += |r| e) around an inner CG on the normal
 * equations whose operator and vectors are FP32 (BF16: links and spinors stored
 * in bfloat16), run to the relative residual max(inner_res, res |b| / (2 |r|)).
 * b, x: F64 full fields (device).  stats may be NULL.  b = 0: x = 0, QXD_OK,
 * no iteration, residual 0 (the same in every solver below). */
qxd_status qxd_solve_cg(qxd_handle *h, const qxd_solver_params *params, void *x, const void *b,
                        qxd_solver_stats *stats, void *stream);

/* Solve D x = b with flexible GCR on D_hat (restart nkv).  With inner_prec F64 a
 * plain FP64 FGCR; with F32 or BF16 an FP64 defect-correction loop around an
 * inner FGCR whose operator and vectors are FP32 (BF16: links and spinors stored
 * in bfloat16).  net: NULL or a network preconditioner M(r) = |r| N(r/|r|) used
 * inside the inner FGCR, dropped (stats->fell_back = 1) if its directions are
 * non-finite or the residual stalls for fallback_after steps. */
qxd_status qxd_solve_fgcr(qxd_handle *h, const qxd_solver_params *params, qxd_nn *net, void *x, const void *b,
                          qxd_solver_stats *stats, void *stream);
/* FGCR as qxd_solve_fgcr, preconditioned by deflation with SAP (qxd_dfl_apply):
 * params->sap_ncy (>= 1), sap_nmr, sap_plain for the SAP part and
 * params->dfl_nc coarse steps; FP32 or bf16-link inner solves.
 * stats->sap_applies counts the preconditioner applications. */
qxd_status qxd_solve_fgcr_dfl(qxd_handle *h, const qxd_solver_params *params, qxd_dfl *dfl, void *x,
                              const void *b, qxd_solver_stats *stats, void *stream);

/* SAP, the paper's Schwarz alternating procedure preconditioner (Sec. 4.4,
 * SAP+GCR), applied to the Schur system: out_e = (M (in_e, 0))_e, where M is
 * ncy cycles of SAP on the full operator D in FP32 from x = 0.  The extended
 * lattice is cut into 4^4 blocks coloured by the parity of their block
 * coordinates; a cycle visits colour 0 then colour 1 and, on every block of
 * that colour, takes the residual r = eta - D x, solves D_B e = r_B
 * approximately, D_B being D restricted to the block (hops leaving it
 * dropped), and adds e to x.  The block solve is nmr minimal-residual steps
 * from e = 0: with eo = 1 (the paper's choice) on the block's even-odd Schur
 * complement H_ee - D_eo H_oo^-1 D_oe with source r_e - D_eo H_oo^-1 r_o, then
 * e_o = H_oo^-1 (r_o - D_oe e_e); with eo = 0 on D_B itself.  (Exact block
 * elimination would make out_e = D_hat^-1 in_e.)  in_e, out_e: FP32 even half
 * fields (device, distinct).  The library keeps block-ordered copies of the
 * links and clover blocks (about 680 bytes a site of the extended lattice)
 * until qxd_trim or qxd_destroy.  QXD_EGEOM unless every extended extent is a
 * multiple of 8 and, with C* in k >= 2, L1 is a multiple of 8; QXD_EINVAL for
 * ncy or nmr outside 1..64 or eo not 0 or 1; QXD_ESTATE before the clover
 * inverse.  Also the FGCR preconditioner (qxd_solver_params.sap_ncy). */
qxd_status qxd_sap_apply(qxd_handle *h, int ncy, int nmr, int eo, void *out_e, const void *in_e, void *stream);
/* The same SAP on full FP32 fields (even half, then odd half, 12 Ve complex64):
 * out = M in with in nonzero on both parities; in, out distinct. */
qxd_status qxd_sap_apply_full(qxd_handle *h, int ncy, int nmr, int eo, void *out, const void *in, void *stream);

/* ---------------------------------------------------------------------------
 * Inexact deflation (the paper's DFL+SAP+GCR, Sec. 4.4), FP32.  A deflation
 * subspace of ns vectors is made rich in low modes by approximate inverse
 * iteration (v <- M_sap v / |M_sap v|, plain SAP block solves), cut into the 4^4
 * SAP blocks and orthonormalised block by block (basis W); the little operator
 * A = W^+ D W couples a block to itself and its 8 face neighbours.  The
 * preconditioner is psi + M_sap (eta - D psi), psi = W c with c from nc GCR
 * steps on A c = W^+ eta (an inexact coarse solve).  A subspace belongs to the
 * operator it was made with: one per quark charge (qxd_dfl_little rebuilds A for
 * another operator from the same basis).  The geometry must admit SAP
 * (QXD_EGEOM otherwise).
 */
#define QXD_DFL_MAXNS 24
#define QXD_DFL_MAXNC 32

/* A deflation object for the handle's lattice: basis, little operator and work
 * fields (96 ns + 192 bytes per extended site and 72 ns^2 bytes per block);
 * ns in 1..QXD_DFL_MAXNS.  It may serve any handle of the same lattice
 * (QXD_EINVAL for another lattice); the little operator belongs to the handle
 * and operator it was last built with (qxd_dfl_generate, qxd_dfl_little). */
qxd_status qxd_dfl_create(qxd_handle *h, int ns, qxd_dfl **d);
qxd_status qxd_dfl_destroy(qxd_dfl *d);
/* Build the subspace from ns start vectors v (FP32 full fields, contiguous,
 * 12 Ve complex64 each, device; overwritten with the vectors after nit rounds
 * of inverse iteration with ncy SAP cycles of nmr steps), then the basis and the
 * little operator for the handle's current operator.  QXD_ESTATE before the
 * clover inverse; QXD_EINVAL for nit outside 0..100 or bad SAP parameters. */
qxd_status qxd_dfl_generate(qxd_handle *h, qxd_dfl *d, void *v, int nit, int ncy, int nmr, void *stream);
/* Rebuild the little operator for the handle's current operator (after a new
 * flavour or gauge field) from the same basis. */
qxd_status qxd_dfl_little(qxd_handle *h, qxd_dfl *d, void *stream);
/* The preconditioner of the Schur system: out_e = (M (in_e, 0))_e with nc
 * coarse GCR steps (1..QXD_DFL_MAXNC) and ncy SAP cycles of nmr steps (eo as in
 * qxd_sap_apply); FP32 even half fields, distinct.  QXD_ESTATE when the little
 * operator was built for another handle or an earlier operator of this one. */
qxd_status qxd_dfl_apply(qxd_handle *h, qxd_dfl *d, int nc, int ncy, int nmr, int eo, void *out_e,
                         const void *in_e, void *stream);
/* Basis vector k of every block as one FP32 full field (device). */
qxd_status qxd_dfl_basis(qxd_handle *h, qxd_dfl *d, int k, void *out, void *stream);
/* Copy the little operator (nblk * 9 * ns * ns complex64, [block][n][k][l]: entry
 * (w_{block,l}, D w_{neighbour n,k})) and
 * the neighbour table (nblk * 9 ints; n = 0 the block, 1 + 2 mu its +mu and
 * 2 + 2 mu its -mu neighbour) to host memory.  Blocks are numbered colour-major
 * (all blocks of even block-coordinate parity first, x3 fastest). */
qxd_status qxd_dfl_little_get(qxd_dfl *d, float *A, int *nbr);
qxd_status qxd_dfl_size(const qxd_dfl *d, int *nblk, int *ns);

/* ---------------------------------------------------------------------------
 * Shifted normal solves and the RHMC rational operator (App. A of the paper;
 * the MSCG solver of its sample input, App. C).  M = D_hat^+ D_hat on the even
 * sites; FP64 throughout.  Of the solver parameters these read nmx (iteration
 * limit), res (relative residual asked of every shifted system) and
 * check_every (iterations between the host's convergence checks).
 */
#define QXD_MS_MAXSHIFT 24

/* Multi-shift CG: x_e[j] = (M + shifts[j])^-1 b_e for j < nshift, all from one
 * Krylov space (CG on the smallest shift, the others by the shifted-CG scalar
 * recurrences; a shift stops once its residual is below res |b_e|).  With the
 * shifts mu^2 these are the twisted-mass normal solves (D_hat^+ D_hat + mu^2).
 * shifts: host array of nshift values >= 0; x_e: host array of nshift device
 * pointers to distinct FP64 even half fields (caller-owned, overwritten);
 * b_e: FP64 even half field, not one of x_e.  stats->inner_it: iterations;
 * stats->true_residual: the largest |b - (M + s_j) x_j| / |b| recomputed at the
 * end; stats->schur_applies: D_hat and D_hat^+ applications.  b_e = 0: every
 * x_e[j] = 0, QXD_OK.  The library holds nshift + 3 FP64 half fields of workspace.  QXD_EINVAL for nshift outside
 * 1..QXD_MS_MAXSHIFT, a negative or non-finite shift, aliased or NULL fields;
 * QXD_ESTATE before the clover inverse; QXD_ENOCONV when nmx iterations do not
 * reach res; QXD_ENAN on a non-finite residual. */
qxd_status qxd_solve_mscg(qxd_handle *h, const qxd_solver_params *prm, int nshift, const double *shifts,
                          void *const *x_e, const void *b_e, qxd_solver_stats *stats, void *stream);

/* The rational operator out_e = A prod_{j<n} (M + nu_j^2) (M + mu_j^2)^-1 in_e
 * (App. A.1), evaluated by partial fractions, A (1 + sum_j sigma_j
 * (M + mu_j^2)^-1) with sigma_j = (nu_j^2 - mu_j^2) prod_{m != j} (nu_m^2 -
 * mu_j^2) / (mu_m^2 - mu_j^2) (App. A.2), and one multi-shift solve whose
 * solutions are summed as they converge (never stored).  A factor P_{k,l} of a
 * frequency-split approximation is the call with A = 1 and the sub-arrays
 * nu + k, mu + k, n = l - k + 1.  nu, mu: host arrays, the mu_j^2 distinct;
 * in_e, out_e: FP64 even half fields (may alias; in_e = 0 gives out_e = 0).
 * stats->true_residual: the largest recurrence residual |zeta_j r| / |in| of the
 * shifted systems at their last update (not recomputed).  Errors as qxd_solve_mscg, and QXD_EINVAL for
 * repeated mu_j^2. */
qxd_status qxd_rational_apply(qxd_handle *h, const qxd_solver_params *prm, double A, int n, const double *nu,
                              const double *mu, void *out_e, const void *in_e, qxd_solver_stats *stats,
                              void *stream);

/* ---------------------------------------------------------------------------
 * Learned preconditioner: three 3^4-tap convolutions on the extended lattice
 * whose taps follow the C* neighbour map (x + d is a composition of unit steps),
 * real channels 24 -> 32 -> 32 -> 24, no biases, ReLU after layers 1 and 2.
 * Input: an even half spinor embedded on the full lattice with zero odd sites
 * (channel 2c = Re, 2c+1 = Im of component c); output kept on the even sites.
 * Weights: FP32 master copy, layers packed one after another, each
 * [81 taps][cout][cin] with tap = 27(d0+1) + 9(d1+1) + 3(d2+1) + (d3+1);
 * 207,360 floats in total.  Activations are stored in bfloat16; the
 * contractions run on MFMA with bfloat16 operands and FP32 accumulation. */

#define QXD_NN_NWEIGHTS 207360

typedef struct {
  int epochs;
  int batch;
  double lr;           /* Adam step size */
  double beta1, beta2, eps;
  int holdout;         /* the last `holdout` pairs are not trained on */
  uint64_t seed;       /* shuffling order */
  int loss;            /* 0: |N(rhat) - ehat|^2 / |ehat|^2;
                          1: |D_hat (N(rhat) - ehat)|^2 / |rhat|^2 (rhat = D_hat ehat):
                             the same error measured in the D_hat^+ D_hat norm, i.e.
                             the residual left after one preconditioned step */
} qxd_train_params;

typedef struct {
  double loss_first;   /* mean training loss of the first epoch */
  double loss_last;    /* mean training loss of the last epoch */
  double holdout_loss; /* mean loss on the held-out pairs after training */
  double t_ms;
  int64_t steps;
} qxd_train_stats;

qxd_status qxd_nn_create(qxd_handle *h, qxd_nn **net);
qxd_status qxd_nn_destroy(qxd_nn *net);
/* Linear skip: M(r) = |r| (N(r/|r|) + skip r/|r|) (default 0: the plain network).
 * A bias-free ReLU network of these widths cannot represent a linear map of 24
 * channels; with a skip it learns a correction to skip * identity. */
qxd_status qxd_nn_set_skip(qxd_nn *net, double skip);
/* Host pointers to QXD_NN_NWEIGHTS floats (synchronous). */
qxd_status qxd_nn_set_weights(qxd_nn *net, const float *w);
qxd_status qxd_nn_get_weights(qxd_nn *net, float *w);

/* Save the network (FP32 master weights and the skip coefficient) to a file,
 * or load one saved by qxd_nn_save into `net` (Adam state reset, as
 * qxd_nn_set_weights).  The file holds an 8-byte tag, the weight count, the
 * skip, an FNV-1a hash of the weight bytes, then the weights in the packed
 * order above.  Synchronous.  QXD_EIO if the file cannot be written or read,
 * or its tag, count, length or hash does not match. */
qxd_status qxd_nn_save(qxd_nn *net, const char *path);
qxd_status qxd_nn_load(qxd_nn *net, const char *path);

/* out_e = |in_e| N(in_e / |in_e|): F32 even half fields. */
qxd_status qxd_nn_apply(qxd_handle *h, qxd_nn *net, void *out_e, const void *in_e, void *stream);

/* Loss and FP32 weight gradient (host, QXD_NN_NWEIGHTS floats) over a batch of
 * pairs: mean_i of the loss selected by loss_kind (see qxd_train_params.loss) with
 * rhat = r_i/|r_i|, ehat = e_i/|r_i|.  r, e: device arrays of n F32 even half
 * fields, one after another.  Synchronous. */
qxd_status qxd_nn_loss_grad(qxd_handle *h, qxd_nn *net, const void *r, const void *e, int n, int loss_kind,
                            double *loss, float *grad, void *stream);

/* Harvest training pairs from an FP64 GCR solve of D_hat x = bhat (no
 * preconditioner): the residuals r_k and errors e_k = x* - x_k at npairs steps
 * spread over the solve, stored as F32 even half fields in r_out, e_out (device,
 * npairs fields each).  b: F64 full field. */
qxd_status qxd_nn_harvest(qxd_handle *h, const void *b, int npairs, void *r_out, void *e_out,
                          int *n_harvested, void *stream);

/* Adam training on pairs (r, e) as above, all taken on the handle's current
 * gauge field and flavour (loss 1 applies that D_hat); synchronous.  Training on
 * several fields is a loop over fields, one call per field and pass: the Adam
 * state persists in the network between calls. */
qxd_status qxd_nn_train(qxd_handle *h, qxd_nn *net, const qxd_train_params *p, const void *r, const void *e,
                        int npairs, qxd_train_stats *stats, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* QXD_H */
