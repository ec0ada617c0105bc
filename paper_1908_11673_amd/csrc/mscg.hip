// Multi-shift conjugate gradients on the normal Schur operator and the RHMC
// rational operator built on it (App. A of arXiv:1908.11673; the MSCG solver
// of its sample input, App. C), in FP64.
//
// One Krylov space serves every shifted system (M + s_j) x_j = phi,
// M = D_hat^+ D_hat: CG runs on the smallest shift s_0 (the slowest system) and
// each other system follows from the same residuals through the scalar
// recurrences of shifted CG,
//   zeta_j(k+1) = zeta_j(k) zeta_j(k-1) a(k-1) /
//                 (a(k) b(k-1) (zeta_j(k-1) - zeta_j(k)) + zeta_j(k-1) a(k-1) (1 + (s_j - s_0) a(k))),
//   a_j(k) = a(k) zeta_j(k+1) / zeta_j(k),  b_j(k) = b(k) (zeta_j(k+1) / zeta_j(k))^2,
//   x_j += a_j p_j,  p_j = zeta_j(k+1) r + b_j p_j,
// with a, b the CG coefficients of the base system; the residual of system j
// is zeta_j r.  A shift stops updating once |zeta_j r| <= res |phi|.
//
// The rational operator R = A prod_j (M + nu_j^2) / (M + mu_j^2) (App. A.1) is
// A (1 + sum_j sigma_j (M + mu_j^2)^-1) by partial fractions (App. A.2), so one
// multi-shift solve on the shifts mu_j^2 gives R phi; the solutions are never
// stored: y += sigma_j a_j p_j accumulates their weighted sum as they grow.
//
// Per iteration: D_hat and D_hat^+ (the cost of a CG step), one pass that
// updates r, one pass that reads r once and every active p_j (and x_j), and two
// one-wavefront kernels for the scalars; the host reads the number of active
// shifts every check_every iterations and never waits otherwise.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "blas.hpp"

namespace {

using clk = std::chrono::steady_clock;

constexpr int kMsMax = QXD_MS_MAXSHIFT;

// device scalar slots (after the network's)
enum {
  S_MS = 3616,
  MS_RR = S_MS,  // |r|^2
  MS_RRN,        // |r_new|^2
  MS_DD,         // |D_hat p|^2
  MS_PP,         // |p|^2 of the base system
  MS_ALPHA,      // a(k)
  MS_AP,         // a(k-1)
  MS_BP,         // b(k-1)
  MS_BETA,       // b(k)
  MS_S0,         // base shift
  MS_TOL2,       // (res |phi|)^2
  MS_NACT,       // shifts still updating
  MS_Z = S_MS + 16,  // zeta_j(k), then zeta_j(k+1) after the beta kernel
  MS_ZP = MS_Z + kMsMax,
  MS_ZN = MS_ZP + kMsMax,
  MS_AJ = MS_ZN + kMsMax,
  MS_BJ = MS_AJ + kMsMax,
  MS_DS = MS_BJ + kMsMax,    // s_j - s_0
  MS_ACT = MS_DS + kMsMax,   // 1 while x_j is updated in this iteration
  MS_ACTN = MS_ACT + kMsMax, // the same for the next iteration
  MS_C = MS_ACTN + kMsMax,   // weight of x_j in the accumulated sum (rational mode)
  MS_RJ = MS_C + kMsMax,     // |zeta_j r|^2 at the shift's last update
  MS_END = MS_RJ + kMsMax
};
static_assert(MS_END <= QXD_NSCAL - 8, "scalar slots");

// workspace roles, the same table as the solvers': 0 source copy, 2 r, 3 D_hat p,
// 5 w, 1 accumulated sum; 16 + j the direction of shift j
enum { W_MS_B = 0, W_MS_Y = 1, W_MS_R = 2, W_MS_T = 3, W_MS_W = 5, W_MS_P = 16 };

struct VecPtrs {
  double2* p[kMsMax];
};

// a(k) and the zeta_j(k+1), a_j(k) of the shifts still active
__global__ void k_ms_alpha(double* __restrict__ scal, int n) {
  const int j = threadIdx.x;
  const double rr = scal[MS_RR];
  const double alpha = rr / (scal[MS_DD] + scal[MS_S0] * scal[MS_PP]);
  const double ap = scal[MS_AP], bp = scal[MS_BP];
  if (j < n) {
    const double act = scal[MS_ACTN + j];
    scal[MS_ACT + j] = act;
    if (act != 0.0) {
      const double z = scal[MS_Z + j], zp = scal[MS_ZP + j];
      const double zn = z * zp * ap / (alpha * bp * (zp - z) + zp * ap * (1.0 + scal[MS_DS + j] * alpha));
      scal[MS_ZN + j] = zn;
      scal[MS_AJ + j] = alpha * zn / z;
    }
  }
  if (j == 0) scal[MS_ALPHA] = alpha;
}

// b(k), the b_j(k), convergence of each shift, and the shift of the recurrences
__global__ void k_ms_beta(double* __restrict__ scal, int n) {
  const int j = threadIdx.x;
  const double rr = scal[MS_RR], rrn = scal[MS_RRN];
  const double beta = rrn / rr;
  double still = 0.0;
  if (j < n && scal[MS_ACT + j] != 0.0) {
    const double z = scal[MS_Z + j], zn = scal[MS_ZN + j];
    const double q = zn / z;
    scal[MS_BJ + j] = beta * q * q;
    scal[MS_ZP + j] = z;
    scal[MS_Z + j] = zn;
    scal[MS_RJ + j] = zn * zn * rrn;
    still = zn * zn * rrn > scal[MS_TOL2] ? 1.0 : 0.0;
    scal[MS_ACTN + j] = still;
  }
  // one wavefront: count the shifts that go on
  for (int off = 32; off > 0; off >>= 1) still += __shfl_xor(still, off);
  __syncthreads();
  if (j == 0) {
    scal[MS_NACT] = still;
    scal[MS_AP] = scal[MS_ALPHA];
    scal[MS_BP] = beta;
    scal[MS_BETA] = beta;
    scal[MS_RR] = rrn;
  }
}

// r -= a (w + s_0 p); partial |r|^2
__global__ __launch_bounds__(QXD_BLOCK) void k_ms_r(double2* __restrict__ r, const double2* __restrict__ w,
                                                    const double2* __restrict__ p, size_t n,
                                                    const double* __restrict__ scal, double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  const double a = scal[MS_ALPHA], s0 = scal[MS_S0];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 wi = ld_stream(&w[i]), pi = ld_stream(&p[i]);
    double2 ri = ld_stream(&r[i]);
    ri.x -= a * (wi.x + s0 * pi.x);
    ri.y -= a * (wi.y + s0 * pi.y);
    st_stream(&r[i], ri);
    acc += ri.x * ri.x + ri.y * ri.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < QXD_BLOCK / 64; ++k) t += sh[k];
    partial[blockIdx.x] = t;
  }
}

// The shifts' vectors are addressed through pointers kept in LDS, which the
// compiler cannot prove global: through a generic pointer the accesses would
// become flat ones, which also count against the LDS wait counter, so every
// read of a coefficient from LDS would wait for the vector loads in flight.
// These helpers address them as global memory (non-temporal, as ld_stream).
typedef __attribute__((address_space(1))) nt_d2 gl_nt_d2;
__device__ inline double2 ld_shift(const double2* p) {
  nt_d2 v = __builtin_nontemporal_load((const gl_nt_d2*)p);
  return make_double2(v.x, v.y);
}
__device__ inline void st_shift(double2* p, double2 a) {
  nt_d2 v = {a.x, a.y};
  __builtin_nontemporal_store(v, (gl_nt_d2*)p);
}

// For every shift: x_j += a_j p_j (ACC: y += c_j a_j p_j instead), then
// p_j = zeta_j r + b_j p_j while x_j is still updated; the base direction is
// always advanced (p = r + b p).  Partial |p_base|^2.
template <bool ACC>
__global__ __launch_bounds__(QXD_BLOCK) void k_ms_update(VecPtrs P, VecPtrs X, double2* __restrict__ y,
                                                         const double2* __restrict__ r, int n, int base, size_t len,
                                                         const double* __restrict__ scal,
                                                         double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  __shared__ double coef[4][kMsMax];  // a_j (or c_j a_j), zeta_j, b_j, flags
  __shared__ double2* pp[kMsMax];     // the pointers, indexed at run time
  __shared__ double2* xp[kMsMax];
  if (threadIdx.x < n) {
    const int j = threadIdx.x;
    pp[j] = P.p[j];
    xp[j] = ACC ? nullptr : X.p[j];
    const bool act = scal[MS_ACT + j] != 0.0;
    const bool adv = act || j == base;
    coef[0][j] = act ? (ACC ? scal[MS_C + j] : 1.0) * scal[MS_AJ + j] : 0.0;
    coef[1][j] = j == base ? 1.0 : scal[MS_Z + j];
    coef[2][j] = j == base ? scal[MS_BETA] : scal[MS_BJ + j];
    coef[3][j] = (act ? 1.0 : 0.0) + (adv ? 2.0 : 0.0);
  }
  __syncthreads();
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (size_t)gridDim.x * blockDim.x) {
    const double2 ri = ld_stream(&r[i]);
    double2 yi = make_double2(0.0, 0.0);
    if (ACC) yi = ld_stream(&y[i]);
    for (int j = 0; j < n; ++j) {
      const double flags = coef[3][j];
      if (flags == 0.0) continue;
      double2 pj = ld_shift(&pp[j][i]);
      if (flags == 1.0 || flags == 3.0) {
        const double a = coef[0][j];
        if (ACC) {
          yi.x += a * pj.x;
          yi.y += a * pj.y;
        } else {
          double2 xj = ld_shift(&xp[j][i]);
          xj.x += a * pj.x;
          xj.y += a * pj.y;
          st_shift(&xp[j][i], xj);
        }
      }
      if (flags >= 2.0) {
        const double z = coef[1][j], b = coef[2][j];
        pj.x = z * ri.x + b * pj.x;
        pj.y = z * ri.y + b * pj.y;
        st_shift(&pp[j][i], pj);
        if (j == base) acc += pj.x * pj.x + pj.y * pj.y;
      }
    }
    if (ACC) st_stream(&y[i], yi);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < QXD_BLOCK / 64; ++k) t += sh[k];
    partial[blockIdx.x] = t;
  }
}

// out = A (phi + y)
__global__ __launch_bounds__(QXD_BLOCK) void k_ms_finish(double2* __restrict__ out, const double2* __restrict__ phi,
                                                         const double2* __restrict__ y, double A, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 a = phi[i], b = y[i];
    out[i] = make_double2(A * (a.x + b.x), A * (a.y + b.y));
  }
}

// r = phi - (M + s) x; partial |r|^2
__global__ __launch_bounds__(QXD_BLOCK) void k_ms_resid(double2* __restrict__ r, const double2* __restrict__ phi,
                                                        const double2* __restrict__ w, const double2* __restrict__ x,
                                                        double s, size_t n, double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double acc = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double2 a = phi[i], b = w[i], c = x[i];
    const double2 v = make_double2(a.x - b.x - s * c.x, a.y - b.y - s * c.y);
    r[i] = v;
    acc += v.x * v.x + v.y * v.y;
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < QXD_BLOCK / 64; ++k) t += sh[k];
    partial[blockIdx.x] = t;
  }
}

qxd_status read_slots(qxd_handle* h, int first, int count, hipStream_t s) {
  QXD_HIP(hipMemcpyAsync(h->scal_host + first, h->scal + first, count * sizeof(double), hipMemcpyDeviceToHost, s));
  QXD_HIP(hipStreamSynchronize(s));
  return QXD_OK;
}

// The multi-shift iteration.  X: the solutions (mscg) or nullptr (rational
// mode: y accumulates sum_j c_j x_j).  Returns the iteration count in *iters.
qxd_status ms_run(qxd_handle* h, const qxd_solver_params* prm, int n, const double* shifts, const double* c,
                  double2* const* X, double2* y, const double2* phi, double nphi, qxd_solver_stats* st,
                  hipStream_t s) {
  const size_t len = (size_t)12 * h->Ve, bytes = len * sizeof(double2);
  double2* r = (double2*)ws_get(h, W_MS_R, bytes);
  double2* t = (double2*)ws_get(h, W_MS_T, bytes);
  double2* w = (double2*)ws_get(h, W_MS_W, bytes);
  if (!r || !t || !w) return QXD_ENOMEM;
  VecPtrs P{}, XP{};
  for (int j = 0; j < n; ++j) {
    P.p[j] = (double2*)ws_get(h, W_MS_P + j, bytes);
    if (!P.p[j]) return QXD_ENOMEM;
    QXD_HIP(hipMemcpyAsync(P.p[j], phi, bytes, hipMemcpyDeviceToDevice, s));
    if (X) {
      XP.p[j] = X[j];
      blas_zero<double2>(X[j], len, s);
    }
  }
  if (y) blas_zero<double2>(y, len, s);
  QXD_HIP(hipMemcpyAsync(r, phi, bytes, hipMemcpyDeviceToDevice, s));
  const int base = (int)(std::min_element(shifts, shifts + n) - shifts);
  // initial scalars: zeta = zeta_prev = 1, a(-1) = 1, b(-1) = 0, every shift active
  double* hs = h->scal_host;
  for (int j = 0; j < n; ++j) {
    hs[MS_Z + j] = hs[MS_ZP + j] = 1.0;
    hs[MS_DS + j] = shifts[j] - shifts[base];
    hs[MS_ACTN + j] = hs[MS_ACT + j] = 1.0;
    hs[MS_C + j] = c ? c[j] : 1.0;
    hs[MS_ZN + j] = hs[MS_AJ + j] = hs[MS_BJ + j] = 0.0;
    hs[MS_RJ + j] = nphi * nphi;
  }
  hs[MS_RR] = hs[MS_PP] = nphi * nphi;
  hs[MS_AP] = 1.0;
  hs[MS_BP] = 0.0;
  hs[MS_S0] = shifts[base];
  hs[MS_TOL2] = (prm->res * nphi) * (prm->res * nphi);
  hs[MS_NACT] = n;
  QXD_HIP(hipMemcpyAsync(h->scal + S_MS, hs + S_MS, (MS_END - S_MS) * sizeof(double), hipMemcpyHostToDevice, s));
  const int check = prm->check_every > 0 ? prm->check_every : 1;
  int it = 0;
  qxd_status rc = QXD_ENOCONV;
  while (true) {
    if (it % check == 0) {
      QXD_TRY(read_slots(h, MS_RR, MS_NACT - MS_RR + 1, s));
      if (!std::isfinite(hs[MS_RR])) { rc = QXD_ENAN; break; }
      if (hs[MS_NACT] == 0.0) { rc = QXD_OK; break; }
    }
    if (it >= prm->nmx) break;
    // w = M p_base, |D_hat p|^2
    QXD_TRY(qxd_schur_apply(h, QXD_F64, 0, t, P.p[base], h->scal + MS_DD, s));
    QXD_TRY(qxd_schur_apply(h, QXD_F64, 1, w, t, nullptr, s));
    st->schur_applies += 2;
    hipLaunchKernelGGL(k_ms_alpha, dim3(1), dim3(64), 0, s, h->scal, n);
    hipLaunchKernelGGL(k_ms_r, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, r, w, P.p[base], len, h->scal, h->partial);
    launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, h->scal + MS_RRN, s);
    hipLaunchKernelGGL(k_ms_beta, dim3(1), dim3(64), 0, s, h->scal, n);
    if (y)
      hipLaunchKernelGGL(k_ms_update<true>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, P, XP, y, r, n, base, len,
                         h->scal, h->partial);
    else
      hipLaunchKernelGGL(k_ms_update<false>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, P, XP, y, r, n, base, len,
                         h->scal, h->partial);
    launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, h->scal + MS_PP, s);
    QXD_HIP(hipGetLastError());
    ++it;
  }
  st->inner_it = it;
  st->outer_it = 1;
  // the largest recurrence residual |zeta_j r| / |phi| at each shift's last update
  QXD_TRY(read_slots(h, MS_RJ, n, s));
  double worst = 0.0;
  for (int j = 0; j < n; ++j) worst = std::max(worst, hs[MS_RJ + j]);
  st->true_residual = std::sqrt(worst) / nphi;
  return rc;
}

qxd_status ms_check(qxd_handle* h, const qxd_solver_params* prm, int n) {
  if (!prm || prm->nmx < 1 || !(prm->res > 0.0)) return QXD_EINVAL;
  if (n < 1 || n > kMsMax) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  return QXD_OK;
}

qxd_status ms_norm(qxd_handle* h, const double2* phi, double* nphi, hipStream_t s) {
  blas_norm2<double2>(h, phi, (size_t)12 * h->Ve, h->scal + MS_RR, s);
  QXD_TRY(read_slots(h, MS_RR, 1, s));
  *nphi = std::sqrt(h->scal_host[MS_RR]);
  if (!std::isfinite(*nphi)) return QXD_ENAN;
  return QXD_OK;
}

// phi = 0: every shifted solution, and R phi, vanish exactly; no iteration.
qxd_status ms_zero(qxd_handle* h, int n, double2* const* out, qxd_solver_stats* stats, clk::time_point t0,
                   hipStream_t s) {
  for (int j = 0; j < n; ++j) blas_zero<double2>(out[j], (size_t)12 * h->Ve, s);
  QXD_HIP(hipGetLastError());
  QXD_HIP(hipStreamSynchronize(s));
  qxd_solver_stats st{};
  st.status = QXD_OK;
  st.true_residual = 0.0;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return QXD_OK;
}

}  // namespace

extern "C" qxd_status qxd_solve_mscg(qxd_handle* h, const qxd_solver_params* prm, int nshift, const double* shifts,
                                     void* const* x_e, const void* b_e, qxd_solver_stats* stats, void* stream) {
  auto t0 = clk::now();
  if (!h || !shifts || !x_e || !b_e) return QXD_EINVAL;
  QXD_TRY(ms_check(h, prm, nshift));
  for (int j = 0; j < nshift; ++j) {
    if (!x_e[j] || x_e[j] == b_e || !std::isfinite(shifts[j]) || shifts[j] < 0.0) return QXD_EINVAL;
    for (int k = 0; k < j; ++k)
      if (x_e[k] == x_e[j]) return QXD_EINVAL;
  }
  hipStream_t s = as_stream(stream);
  const double2* phi = (const double2*)b_e;
  qxd_solver_stats st{};
  double nphi;
  QXD_TRY(ms_norm(h, phi, &nphi, s));
  double2* const* X = reinterpret_cast<double2* const*>(x_e);
  if (nphi == 0.0) return ms_zero(h, nshift, X, stats, t0, s);
  qxd_status rc = ms_run(h, prm, nshift, shifts, nullptr, X, nullptr, phi, nphi, &st, s);
  if (rc == QXD_OK || rc == QXD_ENOCONV) {
    // true residuals |phi - (M + s_j) x_j| / |phi|, the largest reported
    const size_t len = (size_t)12 * h->Ve, bytes = len * sizeof(double2);
    double2* t = (double2*)ws_get(h, W_MS_T, bytes);
    double2* w = (double2*)ws_get(h, W_MS_W, bytes);
    double2* r = (double2*)ws_get(h, W_MS_R, bytes);
    double worst = 0.0;
    for (int j = 0; j < nshift; ++j) {
      QXD_TRY(qxd_schur_apply(h, QXD_F64, 0, t, X[j], nullptr, s));
      QXD_TRY(qxd_schur_apply(h, QXD_F64, 1, w, t, nullptr, s));
      st.schur_applies += 2;
      hipLaunchKernelGGL(k_ms_resid, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, r, phi, w, X[j], shifts[j], len,
                         h->partial);
      launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, h->scal + MS_RRN, s);
      QXD_TRY(read_slots(h, MS_RRN, 1, s));
      worst = std::max(worst, std::sqrt(h->scal_host[MS_RRN]) / nphi);
    }
    st.true_residual = worst;
    if (rc == QXD_OK && !(worst <= prm->res)) rc = QXD_ENOCONV;
  }
  st.status = rc;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

extern "C" qxd_status qxd_rational_apply(qxd_handle* h, const qxd_solver_params* prm, double A, int n,
                                         const double* nu, const double* mu, void* out_e, const void* in_e,
                                         qxd_solver_stats* stats, void* stream) {
  auto t0 = clk::now();
  if (!h || !nu || !mu || !out_e || !in_e || !std::isfinite(A)) return QXD_EINVAL;
  QXD_TRY(ms_check(h, prm, n));
  // partial fractions of prod_j (x + nu_j^2) / (x + mu_j^2) (App. A.2)
  std::vector<double> shifts(n), sigma(n);
  for (int j = 0; j < n; ++j) {
    if (!std::isfinite(nu[j]) || !std::isfinite(mu[j])) return QXD_EINVAL;
    shifts[j] = mu[j] * mu[j];
  }
  for (int j = 0; j < n; ++j) {
    double sg = nu[j] * nu[j] - shifts[j];
    for (int m = 0; m < n; ++m) {
      if (m == j) continue;
      if (!(shifts[m] != shifts[j])) return QXD_EINVAL;  // the poles must be distinct
      sg *= (nu[m] * nu[m] - shifts[j]) / (shifts[m] - shifts[j]);
    }
    sigma[j] = sg;
  }
  hipStream_t s = as_stream(stream);
  const double2* phi = (const double2*)in_e;
  const size_t len = (size_t)12 * h->Ve, bytes = len * sizeof(double2);
  double2* y = (double2*)ws_get(h, W_MS_Y, bytes);
  double2* keep = (double2*)ws_get(h, W_MS_B, bytes);
  if (!y || !keep) return QXD_ENOMEM;
  if (out_e == in_e) {  // the source is read again at the end
    QXD_HIP(hipMemcpyAsync(keep, phi, bytes, hipMemcpyDeviceToDevice, s));
    phi = keep;
  }
  qxd_solver_stats st{};
  double nphi;
  QXD_TRY(ms_norm(h, phi, &nphi, s));
  if (nphi == 0.0) {
    double2* o = (double2*)out_e;
    return ms_zero(h, 1, &o, stats, t0, s);
  }
  qxd_status rc = ms_run(h, prm, n, shifts.data(), sigma.data(), nullptr, y, phi, nphi, &st, s);
  if (rc == QXD_OK || rc == QXD_ENOCONV)
    hipLaunchKernelGGL(k_ms_finish, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, (double2*)out_e, phi, y, A, len);
  QXD_HIP(hipGetLastError());
  QXD_HIP(hipStreamSynchronize(s));
  st.status = rc;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}
