// Krylov solvers on the even-odd preconditioned operator D_hat (Sec. 2.3 and
// 4.4 of arXiv:1908.11673): CG on the normal equations in FP64, and flexible
// GCR (optionally with the network preconditioner) inside an FP64
// defect-correction loop whose inner operator and vectors are FP32 (or FP32
// with bfloat16 links).  Every solve ends with the FP64 true residual
// |b - D x| / |b| recomputed on the full lattice.
#include <chrono>
#include <cmath>
#include <complex>
#include <functional>
#include <vector>

#include "blas.hpp"
#include "sap_blocks.hpp"

namespace {

using clk = std::chrono::steady_clock;

// workspace roles
enum {
  W_BH = 0, W_XE, W_R, W_P, W_Z, W_W, W_FULL0, W_FULL1,  // FP64 halves (FULL*: full fields)
  W_R32 = 10, W_E32, W_E64,  // 8, 9, 13, 14: SAP's block-order fields (sap.hip)
  W_PHI = 16,    // 16..(16+QXD_MAXKV-1)
  W_CHI = 40     // 40..(40+QXD_MAXKV-1) -> needs ws[] of 64+: keep nkv <= 24
};

qxd_status read_scal(qxd_handle* h, int first, int count, hipStream_t s) {
  QXD_HIP(hipMemcpyAsync(h->scal_host + first, h->scal + first, count * sizeof(double), hipMemcpyDeviceToHost, s));
  QXD_HIP(hipStreamSynchronize(s));
  return QXD_OK;
}

// full-lattice FP64 true relative residual |b - D x| / |b|
qxd_status true_residual(qxd_handle* h, const double2* x, const double2* b, double nb, double* res, hipStream_t s) {
  size_t nfull = (size_t)24 * h->Ve;
  double2* w = (double2*)ws_get(h, W_FULL0, nfull * sizeof(double2));
  if (!w) return QXD_ENOMEM;
  QXD_TRY(qxd_dw_apply(h, QXD_F64, w, x, s));
  blas_sub_norm<double2>(h, nullptr, b, w, nfull, h->scal + S_RT, s);
  QXD_TRY(read_scal(h, S_RT, 1, s));
  *res = std::sqrt(h->scal_host[S_RT]) / nb;
  return QXD_OK;
}

// |b| of a full field; QXD_ENAN if it is not finite.
qxd_status norm_source(qxd_handle* h, const double2* b, double* nb, hipStream_t s) {
  blas_norm2<double2>(h, b, (size_t)24 * h->Ve, h->scal + S_NB, s);
  QXD_TRY(read_scal(h, S_NB, 1, s));
  *nb = std::sqrt(h->scal_host[S_NB]);
  if (!std::isfinite(*nb)) return QXD_ENAN;
  return QXD_OK;
}

// As norm_source, with a vanishing b rejected (QXD_EINVAL).
qxd_status norm_full(qxd_handle* h, const double2* b, double* nb, hipStream_t s) {
  QXD_TRY(norm_source(h, b, nb, s));
  if (*nb == 0.0) return QXD_EINVAL;
  return QXD_OK;
}

// b = 0: x = 0 solves D x = b exactly; no iteration, residual 0.
qxd_status zero_solution(qxd_handle* h, void* x, qxd_solver_stats* stats, clk::time_point t0, hipStream_t s) {
  blas_zero<double2>((double2*)x, (size_t)24 * h->Ve, s);
  QXD_HIP(hipGetLastError());
  QXD_HIP(hipStreamSynchronize(s));
  qxd_solver_stats st{};
  st.status = QXD_OK;
  st.true_residual = 0.0;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return QXD_OK;
}

// The operator of an inner solve.
struct InnerOp {
  int mode;  // 0: FP64, 1: FP32, 2: FP32 vectors with bfloat16 links
};

template <class VT>
qxd_status apply_op(qxd_handle* h, InnerOp op, VT* out, const VT* in, double* norm_slot, hipStream_t s) {
  if (op.mode == 0) return qxd_schur_apply(h, QXD_F64, 0, out, in, norm_slot, s);
  if (op.mode == 1) return qxd_schur_apply(h, QXD_F32, 0, out, in, norm_slot, s);
  return qxd_schur_apply_mixed(h, 0, (float4*)out, (const float4*)in, norm_slot, s);
}

template <class VT>
qxd_status apply_op_dag(qxd_handle* h, InnerOp op, int dagger, VT* out, const VT* in, double* norm_slot,
                        hipStream_t s) {
  if (op.mode == 0) return qxd_schur_apply(h, QXD_F64, dagger, out, in, norm_slot, s);
  if (op.mode == 1) return qxd_schur_apply(h, QXD_F32, dagger, out, in, norm_slot, s);
  return qxd_schur_apply_mixed(h, dagger, (float4*)out, (const float4*)in, norm_slot, s);
}

// CG on the normal equations D_hat^+ D_hat x = D_hat^+ b of the inner operator,
// x from zero; r holds b on entry and the recursive residual b - D_hat x on
// exit.  Stops when |r| <= tol_abs (checked every `check` iterations) or after
// max_steps iterations.  Device scalars: S_ZZ0/1 |z|^2, S_WW |w|^2, S_FRR |r|^2.
template <class VT>
qxd_status cgnr(qxd_handle* h, InnerOp op, VT* x, VT* r, VT* p, VT* z, VT* w, size_t n, double tol_abs,
                int max_steps, int check, int* steps, int64_t* applies, hipStream_t s) {
  const size_t bytes = n * sizeof(VT);
  blas_zero<VT>(x, n, s);
  QXD_TRY(apply_op_dag<VT>(h, op, 1, z, r, h->scal + S_ZZ0, s));
  QXD_HIP(hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, s));
  *applies += 1;
  int it = 0;
  while (it < max_steps) {
    const int zo = S_ZZ0 + (it & 1), zn = S_ZZ0 + ((it + 1) & 1);
    QXD_TRY(apply_op_dag<VT>(h, op, 0, w, p, h->scal + S_WW, s));
    blas_cg_xr<VT>(h, x, r, p, w, n, zo, S_WW, S_FRR, s);
    QXD_TRY(apply_op_dag<VT>(h, op, 1, z, r, h->scal + zn, s));
    blas_cg_p<VT>(h, p, z, n, zn, zo, s);
    *applies += 2;
    ++it;
    if (it % check == 0) {
      QXD_TRY(read_scal(h, S_FRR, 1, s));
      double rr = h->scal_host[S_FRR];
      if (!std::isfinite(rr)) return QXD_ENAN;
      if (std::sqrt(rr) <= tol_abs) break;
    }
  }
  *steps = it;
  return QXD_OK;
}

// The right preconditioner of the inner FGCR: the network or SAP (FP32 only).
struct Precond {
  qxd_nn* net = nullptr;
  int sap_ncy = 0, sap_nmr = 0, sap_eo = 1;
  qxd_dfl* dfl = nullptr;  // deflation: coarse correction, then SAP
  int dfl_nc = 16;
  bool any() const { return net != nullptr || sap_ncy > 0; }
};

template <class VT>
qxd_status precond_apply(qxd_handle* h, const Precond& pc, VT* out, const VT* in, hipStream_t s);
template <>
qxd_status precond_apply<float4>(qxd_handle* h, const Precond& pc, float4* out, const float4* in, hipStream_t s) {
  if (pc.net) return nn_apply_internal(h, pc.net, out, in, s);
  if (pc.dfl) return dfl_apply_internal(h, pc.dfl, pc.dfl_nc, pc.sap_ncy, pc.sap_nmr, pc.sap_eo, out, in, s);
  return sap_apply_internal(h, pc.sap_ncy, pc.sap_nmr, pc.sap_eo, out, in, s);
}
template <>
qxd_status precond_apply<double2>(qxd_handle*, const Precond&, double2*, const double2*, hipStream_t) {
  return QXD_EINVAL;
}

struct FgcrResult {
  int steps = 0;
  int64_t applies = 0;
  int64_t nn_applies = 0;
  int64_t sap_applies = 0;
  bool fell_back = false;
  double rr = 0.0;  // final recursive |r|^2
};

// Flexible GCR on op x = b, x starting at zero; r holds b on entry and the
// recursive residual on exit.  Classical Gram-Schmidt of chi_k against the
// previous directions, normalisation, then r -= (chi_k, r) chi_k; at the end of
// each cycle x += Phi alpha with R alpha = c solved on the host in FP64.  The
// host waits once per step, for |chi_k|^2 and |r|^2 together: a direction whose
// norm is zero or not finite is zeroed by the normalisation, so the residual
// update leaves r as it was and the step can be redone without the
// preconditioner.  Without a preconditioner phi_k = r_k, and the residual
// update of step k writes r_{k+1} to phi_{k+1} as well (phi_0 is a copy).
template <class VT>
qxd_status fgcr(qxd_handle* h, InnerOp op, Precond pc, int fallback_after, VT* x, VT* r, size_t n, int nkv,
                double tol_abs, int max_steps, FgcrResult* res, hipStream_t s,
                const std::function<qxd_status()>* on_cycle = nullptr) {
  std::vector<VT*> phi(nkv), chi(nkv);
  size_t bytes = n * sizeof(VT);
  for (int k = 0; k < nkv; ++k) {
    phi[k] = (VT*)ws_get(h, W_PHI + k, bytes);
    chi[k] = (VT*)ws_get(h, W_CHI + k, bytes);
    if (!phi[k] || !chi[k]) return QXD_ENOMEM;
  }
  blas_zero<VT>(x, n, s);
  blas_norm2<VT>(h, r, n, h->scal + S_FRR, s);
  QXD_TRY(read_scal(h, S_FRR, 1, s));
  double rr = h->scal_host[S_FRR];
  if (!std::isfinite(rr)) return QXD_ENAN;
  bool use_nn = pc.any();
  bool r_in_phi = false;  // phi[k] already holds r (written by the previous residual update)
  double best = std::sqrt(rr);
  int since_best = 0;
  int steps = 0;
  while (std::sqrt(rr) > tol_abs && steps < max_steps) {
    int m = 0;
    for (int k = 0; k < nkv && steps < max_steps; ++k) {
      bool redo = true;
      while (redo) {
        redo = false;
        if (use_nn) {
          QXD_TRY(precond_apply<VT>(h, pc, phi[k], r, s));
          if (pc.net)
            res->nn_applies++;
          else
            res->sap_applies++;
        } else if (k == 0 || !r_in_phi) {
          QXD_HIP(hipMemcpyAsync(phi[k], r, bytes, hipMemcpyDeviceToDevice, s));
        }
        if (k == 0) {
          QXD_TRY(apply_op<VT>(h, op, chi[k], phi[k], h->scal + S_FB + k, s));
        } else {
          QXD_TRY(apply_op<VT>(h, op, chi[k], phi[k], nullptr, s));
          Ptrs bp{};
          for (int j = 0; j < k; ++j) bp.p[j] = chi[j];
          double* col = h->scal + S_FR + 2 * k * QXD_MAXKV_R;
          blas_mdot<VT>(h, bp, k, chi[k], n, col, s);
          blas_mupdate<VT>(h, chi[k], bp, k, col, n, h->scal + S_FB + k, s);
        }
        res->applies++;
        blas_scale_cdot<VT>(h, chi[k], r, n, S_FB + k, h->scal + S_FC + 2 * k, s);
        // plain FGCR: the next step's phi is the new residual
        r_in_phi = !use_nn && k + 1 < nkv;
        blas_r_update<VT>(h, r, chi[k], n, S_FC + 2 * k, h->scal + S_FRR, s, r_in_phi ? phi[k + 1] : nullptr);
        QXD_HIP(hipMemcpyAsync(h->scal_host + S_FB + k, h->scal + S_FB + k, sizeof(double), hipMemcpyDeviceToHost,
                               s));
        QXD_TRY(read_scal(h, S_FRR, 1, s));
        double b2 = h->scal_host[S_FB + k];
        if (!std::isfinite(b2) || !(b2 > 0.0)) {
          // chi_k was zeroed and r is unchanged
          r_in_phi = false;
          if (use_nn) {  // the preconditioner produced a useless direction: drop it, redo the step plainly
            use_nn = false;
            res->fell_back = true;
            redo = true;
            continue;
          }
          return std::isfinite(b2) ? QXD_ENOCONV : QXD_ENAN;
        }
      }
      rr = h->scal_host[S_FRR];
      ++m;
      ++steps;
      if (!std::isfinite(rr)) return QXD_ENAN;
      double rn = std::sqrt(rr);
      if (rn < 0.99 * best) {
        best = rn;
        since_best = 0;
      } else if (use_nn && ++since_best >= fallback_after) {
        use_nn = false;
        res->fell_back = true;
      }
      if (rn <= tol_abs) break;
    }
    // x += sum_k alpha_k phi_k with R alpha = c
    QXD_TRY(read_scal(h, S_FB, m, s));
    QXD_TRY(read_scal(h, S_FC, 2 * m, s));
    QXD_TRY(read_scal(h, S_FR, 2 * m * QXD_MAXKV_R, s));
    std::vector<std::complex<double>> al(m);
    for (int k = m - 1; k >= 0; --k) {
      std::complex<double> v(h->scal_host[S_FC + 2 * k], h->scal_host[S_FC + 2 * k + 1]);
      for (int j = k + 1; j < m; ++j) {
        std::complex<double> a(h->scal_host[S_FR + 2 * (j * QXD_MAXKV_R + k)],
                               h->scal_host[S_FR + 2 * (j * QXD_MAXKV_R + k) + 1]);
        v -= a * al[j];
      }
      al[k] = v / std::sqrt(h->scal_host[S_FB + k]);
    }
    for (int k = 0; k < m; ++k) {
      h->scal_host[S_FAL + 2 * k] = al[k].real();
      h->scal_host[S_FAL + 2 * k + 1] = al[k].imag();
    }
    QXD_HIP(hipMemcpyAsync(h->scal + S_FAL, h->scal_host + S_FAL, 2 * m * sizeof(double), hipMemcpyHostToDevice, s));
    Ptrs pp{};
    for (int j = 0; j < m; ++j) pp.p[j] = phi[j];
    blas_multi_axpy<VT>(h, x, pp, m, h->scal + S_FAL, n, s);
    if (on_cycle) QXD_TRY((*on_cycle)());
  }
  res->steps = steps;
  res->rr = rr;
  return QXD_OK;
}

// Default reduction of an inner solve: 1e-5 with the FP32 operator; 1e-3 with
// bfloat16 links and spinors, whose operator differs from the FP64 one by a
// few 1e-3, so that solving it further buys no outer progress (measured: fewer
// inner iterations in total at 64 x 32^3 for CG and FGCR).
double default_inner_res(int inner_prec) { return inner_prec == QXD_BF16 ? 1e-3 : 1e-5; }

qxd_status check_params(const qxd_solver_params* p) {
  if (!p) return QXD_EINVAL;
  if (p->nmx < 1 || !(p->res > 0.0)) return QXD_EINVAL;
  return QXD_OK;
}

// Defect correction around an FP32 (or bfloat16-link) CG: r = bhat - D_hat x in
// FP64; the inner CG solves D_hat e = r / |r| on the normal equations to the
// relative residual max(inner_res, tol / (2 |r|)); x += |r| e in FP64.
qxd_status solve_cg_dc(qxd_handle* h, const qxd_solver_params* prm, void* x, const void* b,
                       qxd_solver_stats* stats, void* stream, clk::time_point t0) {
  hipStream_t s = as_stream(stream);
  size_t n64 = (size_t)12 * h->Ve, n32 = (size_t)6 * h->Ve;
  size_t b64 = n64 * sizeof(double2), b32 = n32 * sizeof(float4);
  double2 *bh = (double2*)ws_get(h, W_BH, b64), *xe = (double2*)ws_get(h, W_XE, b64);
  double2 *r = (double2*)ws_get(h, W_R, b64), *w = (double2*)ws_get(h, W_W, b64);
  float4 *r32 = (float4*)ws_get(h, W_R32, b32), *e32 = (float4*)ws_get(h, W_E32, b32);
  float4 *p32 = (float4*)ws_get(h, W_P, b32), *z32 = (float4*)ws_get(h, W_Z, b32);
  float4* w32 = (float4*)ws_get(h, W_E64, b32);
  if (!bh || !xe || !r || !w || !r32 || !e32 || !p32 || !z32 || !w32) return QXD_ENOMEM;
  qxd_solver_stats st{};
  double nb;
  qxd_status rc = norm_source(h, (const double2*)b, &nb, s);
  if (rc != QXD_OK) return rc;
  if (nb == 0.0) return zero_solution(h, x, stats, t0, s);
  const double tol = prm->res * nb;
  QXD_TRY(qxd_eo_source(h, bh, b, s));
  blas_zero<double2>(xe, n64, s);
  QXD_HIP(hipMemcpyAsync(r, bh, b64, hipMemcpyDeviceToDevice, s));
  blas_norm2<double2>(h, r, n64, h->scal + S_RR, s);
  QXD_TRY(read_scal(h, S_RR, 1, s));
  double rr = h->scal_host[S_RR];
  const int max_outer = prm->max_outer > 0 ? prm->max_outer : 100;
  const double inner_res = prm->inner_res > 0 ? prm->inner_res : default_inner_res(prm->inner_prec);
  const int check = prm->check_every > 0 ? prm->check_every : 1;
  int steps_left = prm->nmx;
  InnerOp op{prm->inner_prec == QXD_F32 ? 1 : 2};
  rc = QXD_ENOCONV;
  for (int outer = 0; outer < max_outer; ++outer) {
    if (!std::isfinite(rr)) { rc = QXD_ENAN; break; }
    double rn = std::sqrt(rr);
    if (rn <= tol) { rc = QXD_OK; break; }
    if (steps_left <= 0) break;
    blas_down(h, r32, r, S_RR, s);
    int steps = 0;
    qxd_status ic = cgnr<float4>(h, op, e32, r32, p32, z32, w32, n32, std::fmax(inner_res, 0.5 * tol / rn),
                                 steps_left, check, &steps, &st.schur_applies, s);
    if (ic != QXD_OK) { rc = ic; break; }
    blas_up_acc(h, xe, e32, S_RR, s);
    st.inner_it += steps;
    steps_left -= steps;
    st.outer_it = outer + 1;
    QXD_TRY(qxd_schur_apply(h, QXD_F64, 0, w, xe, nullptr, s));
    st.schur_applies++;
    blas_sub_norm<double2>(h, r, bh, w, n64, h->scal + S_RR, s);
    QXD_TRY(read_scal(h, S_RR, 1, s));
    rr = h->scal_host[S_RR];
    if (steps == 0 && !(std::sqrt(rr) <= tol)) break;
  }
  if (rc == QXD_OK || rc == QXD_ENOCONV) {
    QXD_TRY(qxd_eo_reconstruct(h, x, xe, b, s));
    QXD_TRY(true_residual(h, (const double2*)x, (const double2*)b, nb, &st.true_residual, s));
    if (rc == QXD_OK && !(st.true_residual <= prm->res)) rc = QXD_ENOCONV;
  }
  st.status = rc;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

}  // namespace

extern "C" qxd_status qxd_solve_cg(qxd_handle* h, const qxd_solver_params* prm, void* x, const void* b,
                                   qxd_solver_stats* stats, void* stream) {
  auto t0 = clk::now();
  if (!h || !x || !b) return QXD_EINVAL;
  QXD_TRY(check_params(prm));
  if (!h->has_inverse) return QXD_ESTATE;
  if (prm->inner_prec == QXD_F32 || prm->inner_prec == QXD_BF16) return solve_cg_dc(h, prm, x, b, stats, stream, t0);
  if (prm->inner_prec != QXD_F64) return QXD_EINVAL;
  hipStream_t s = as_stream(stream);
  size_t n = (size_t)12 * h->Ve;
  size_t bytes = n * sizeof(double2);
  double2 *bh = (double2*)ws_get(h, W_BH, bytes), *xe = (double2*)ws_get(h, W_XE, bytes);
  double2 *r = (double2*)ws_get(h, W_R, bytes), *p = (double2*)ws_get(h, W_P, bytes);
  double2 *z = (double2*)ws_get(h, W_Z, bytes), *w = (double2*)ws_get(h, W_W, bytes);
  if (!bh || !xe || !r || !p || !z || !w) return QXD_ENOMEM;
  qxd_solver_stats st{};
  double nb;
  qxd_status rc = norm_source(h, (const double2*)b, &nb, s);
  if (rc != QXD_OK) return rc;
  if (nb == 0.0) return zero_solution(h, x, stats, t0, s);
  double tol = prm->res * nb;
  QXD_TRY(qxd_eo_source(h, bh, b, s));
  blas_zero<double2>(xe, n, s);
  QXD_HIP(hipMemcpyAsync(r, bh, bytes, hipMemcpyDeviceToDevice, s));
  int check = prm->check_every > 0 ? prm->check_every : 1;
  int it = 0;
  rc = QXD_ENOCONV;
  bool restart = true;
  while (true) {
    if (restart) {
      // z = D^+ r (norm -> zz), p = z, rr = |r|^2
      QXD_TRY(qxd_schur_apply(h, QXD_F64, 1, z, r, h->scal + S_ZZ0 + (it & 1), s));
      st.schur_applies++;
      QXD_HIP(hipMemcpyAsync(p, z, bytes, hipMemcpyDeviceToDevice, s));
      blas_norm2<double2>(h, r, n, h->scal + S_RR, s);
      restart = false;
    }
    if (it % check == 0 || it >= prm->nmx) {
      QXD_TRY(read_scal(h, S_RR, 1, s));
      double rr = h->scal_host[S_RR];
      if (!std::isfinite(rr)) { rc = QXD_ENAN; break; }
      if (std::sqrt(rr) <= tol) {
        // recompute the residual from x
        QXD_TRY(qxd_schur_apply(h, QXD_F64, 0, w, xe, nullptr, s));
        st.schur_applies++;
        blas_sub_norm<double2>(h, r, bh, w, n, h->scal + S_RR, s);
        QXD_TRY(read_scal(h, S_RR, 1, s));
        if (std::sqrt(h->scal_host[S_RR]) <= tol) { rc = QXD_OK; break; }
        restart = true;
        continue;
      }
      if (it >= prm->nmx) break;
    }
    int zo = S_ZZ0 + (it & 1), zn = S_ZZ0 + ((it + 1) & 1);
    QXD_TRY(qxd_schur_apply(h, QXD_F64, 0, w, p, h->scal + S_WW, s));
    blas_cg_xr<double2>(h, xe, r, p, w, n, zo, S_WW, S_RR, s);
    QXD_TRY(qxd_schur_apply(h, QXD_F64, 1, z, r, h->scal + zn, s));
    blas_cg_p<double2>(h, p, z, n, zn, zo, s);
    st.schur_applies += 2;
    ++it;
  }
  st.inner_it = it;
  st.outer_it = 1;
  if (rc == QXD_OK || rc == QXD_ENOCONV) {
    QXD_TRY(qxd_eo_reconstruct(h, x, xe, b, s));
    QXD_TRY(true_residual(h, (const double2*)x, (const double2*)b, nb, &st.true_residual, s));
    if (rc == QXD_OK && !(st.true_residual <= prm->res)) rc = QXD_ENOCONV;
  }
  st.status = rc;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

namespace {

qxd_status solve_fgcr(qxd_handle* h, const qxd_solver_params* prm, qxd_nn* net, qxd_dfl* dfl, void* x,
                      const void* b, qxd_solver_stats* stats, void* stream) {
  auto t0 = clk::now();
  if (!h || !x || !b) return QXD_EINVAL;
  QXD_TRY(check_params(prm));
  if (!h->has_inverse) return QXD_ESTATE;
  int nkv = prm->nkv > 0 ? prm->nkv : 16;
  if (nkv > 24) return QXD_EINVAL;
  int mode = prm->inner_prec == QXD_F64 ? 0 : prm->inner_prec == QXD_F32 ? 1 : prm->inner_prec == QXD_BF16 ? 2 : -1;
  if (mode < 0) return QXD_EINVAL;
  Precond pc;
  pc.net = net;
  if (prm->sap_ncy > 0 || dfl) {
    if (net || prm->sap_ncy < 1 || prm->sap_nmr < 1) return QXD_EINVAL;  // one preconditioner at a time
    if (prm->sap_plain != 0 && prm->sap_plain != 1) return QXD_EINVAL;
    if (prm->dfl_nc < 0 || prm->dfl_nc > QXD_DFL_MAXNC) return QXD_EINVAL;
    if (!sap_supported(h)) return QXD_EGEOM;
    pc.sap_ncy = prm->sap_ncy;
    pc.sap_nmr = prm->sap_nmr;
    pc.sap_eo = 1 - prm->sap_plain;
    pc.dfl = dfl;
    pc.dfl_nc = prm->dfl_nc > 0 ? prm->dfl_nc : 16;
  }
  if (mode == 0 && pc.any()) return QXD_EINVAL;  // the preconditioners run on FP32 vectors
  hipStream_t s = as_stream(stream);
  if (pc.sap_ncy > 0 && !dfl) {
    // the SAP block copies first, while the FP32 odd clover blocks they are
    // made from need not share the memory with the solver's vectors
    const float2* vb;
    const float4* cb;
    SapGeo sb;
    QXD_TRY(sap_blocks(h, pc.sap_eo, &vb, &cb, &sb, s));
  }
  size_t n64 = (size_t)12 * h->Ve, n32 = (size_t)6 * h->Ve;
  size_t b64 = n64 * sizeof(double2);
  double2 *bh = (double2*)ws_get(h, W_BH, b64), *xe = (double2*)ws_get(h, W_XE, b64);
  double2 *r = (double2*)ws_get(h, W_R, b64), *w = (double2*)ws_get(h, W_W, b64);
  double2* e64 = mode == 0 ? (double2*)ws_get(h, W_E64, b64) : nullptr;  // the FP64 FGCR's correction
  if (!bh || !xe || !r || !w || (mode == 0 && !e64)) return QXD_ENOMEM;
  float4 *r32 = nullptr, *e32 = nullptr;
  if (mode != 0) {
    r32 = (float4*)ws_get(h, W_R32, n32 * sizeof(float4));
    e32 = (float4*)ws_get(h, W_E32, n32 * sizeof(float4));
    if (!r32 || !e32) return QXD_ENOMEM;
  }
  qxd_solver_stats st{};
  double nb;
  qxd_status rc = norm_source(h, (const double2*)b, &nb, s);
  if (rc != QXD_OK) return rc;
  if (nb == 0.0) return zero_solution(h, x, stats, t0, s);
  double tol = prm->res * nb;
  QXD_TRY(qxd_eo_source(h, bh, b, s));
  blas_zero<double2>(xe, n64, s);
  QXD_HIP(hipMemcpyAsync(r, bh, b64, hipMemcpyDeviceToDevice, s));
  blas_norm2<double2>(h, r, n64, h->scal + S_RR, s);
  QXD_TRY(read_scal(h, S_RR, 1, s));
  double rr = h->scal_host[S_RR];
  int max_outer = prm->max_outer > 0 ? prm->max_outer : 100;
  double inner_res = prm->inner_res > 0 ? prm->inner_res : default_inner_res(prm->inner_prec);
  int fallback_after = prm->fallback_after > 0 ? prm->fallback_after : 50;
  int steps_left = prm->nmx;
  rc = QXD_ENOCONV;
  InnerOp op{mode};
  for (int outer = 0; outer < max_outer; ++outer) {
    if (!std::isfinite(rr)) { rc = QXD_ENAN; break; }
    double rn = std::sqrt(rr);
    if (rn <= tol) { rc = QXD_OK; break; }
    if (steps_left <= 0) break;
    FgcrResult fr;
    qxd_status ic;
    if (mode == 0) {
      // plain FP64 FGCR on the current residual: D_hat e = r, to the final target
      QXD_HIP(hipMemcpyAsync(w, r, b64, hipMemcpyDeviceToDevice, s));
      ic = fgcr<double2>(h, op, Precond{}, fallback_after, e64, w, n64, nkv, 0.5 * tol, steps_left, &fr, s);
      if (ic != QXD_OK) { rc = ic; break; }
      h->scal_host[S_ONE] = 1.0;
      h->scal_host[S_ONE + 1] = 0.0;
      QXD_HIP(hipMemcpyAsync(h->scal + S_FAL, h->scal_host + S_ONE, 2 * sizeof(double), hipMemcpyHostToDevice, s));
      Ptrs pe{};
      pe.p[0] = e64;
      blas_multi_axpy<double2>(h, xe, pe, 1, h->scal + S_FAL, n64, s);
    } else {
      // FP32 inner solve of D_hat e = r / |r|, then x += |r| e
      blas_down(h, r32, r, S_RR, s);
      double itol = std::fmax(inner_res, 0.5 * tol / rn);
      ic = fgcr<float4>(h, op, pc, fallback_after, e32, r32, n32, nkv, itol, steps_left, &fr, s);
      if (ic != QXD_OK) { rc = ic; break; }
      blas_up_acc(h, xe, e32, S_RR, s);
    }
    st.inner_it += fr.steps;
    st.schur_applies += fr.applies;
    st.nn_applies += fr.nn_applies;
    st.sap_applies += fr.sap_applies;
    st.fell_back |= fr.fell_back ? 1 : 0;
    if (fr.fell_back) pc = Precond{};
    steps_left -= fr.steps;
    st.outer_it = outer + 1;
    // FP64 true residual of the Schur system
    QXD_TRY(qxd_schur_apply(h, QXD_F64, 0, w, xe, nullptr, s));
    st.schur_applies++;
    blas_sub_norm<double2>(h, r, bh, w, n64, h->scal + S_RR, s);
    QXD_TRY(read_scal(h, S_RR, 1, s));
    rr = h->scal_host[S_RR];
    if (fr.steps == 0 && !(std::sqrt(rr) <= tol)) break;
  }
  if (rc == QXD_OK || rc == QXD_ENOCONV) {
    QXD_TRY(qxd_eo_reconstruct(h, x, xe, b, s));
    QXD_TRY(true_residual(h, (const double2*)x, (const double2*)b, nb, &st.true_residual, s));
    if (rc == QXD_OK && !(st.true_residual <= prm->res)) rc = QXD_ENOCONV;
  }
  st.status = rc;
  st.t_ms = std::chrono::duration<double, std::milli>(clk::now() - t0).count();
  if (stats) *stats = st;
  return rc;
}

}  // namespace

extern "C" qxd_status qxd_solve_fgcr(qxd_handle* h, const qxd_solver_params* prm, qxd_nn* net, void* x,
                                     const void* b, qxd_solver_stats* stats, void* stream) {
  return solve_fgcr(h, prm, net, nullptr, x, b, stats, stream);
}

extern "C" qxd_status qxd_solve_fgcr_dfl(qxd_handle* h, const qxd_solver_params* prm, qxd_dfl* dfl, void* x,
                                         const void* b, qxd_solver_stats* stats, void* stream) {
  if (!dfl) return QXD_EINVAL;
  return solve_fgcr(h, prm, nullptr, dfl, x, b, stats, stream);
}

// Training pairs from the method's own solves: plain FP64 GCR (restart 4, no
// preconditioner) on D_hat x = bhat, with the iterate x_k and the recursive
// residual r_k recorded at restarts; after convergence e_k = x* - x_k (formed
// in FP64), so that D_hat e_k = r_k up to the final residual.  npairs snapshots
// evenly spread over the recorded part of the solve are returned as FP32 even
// half fields.
extern "C" qxd_status qxd_nn_harvest(qxd_handle* h, const void* b, int npairs, void* r_out, void* e_out,
                                     int* n_harvested, void* stream) {
  if (!h || !b || npairs < 1 || !r_out || !e_out) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  size_t n64 = (size_t)12 * h->Ve, b64 = n64 * sizeof(double2);
  double2 *bh = (double2*)ws_get(h, W_BH, b64), *xe = (double2*)ws_get(h, W_XE, b64);
  double2 *r = (double2*)ws_get(h, W_R, b64), *w = (double2*)ws_get(h, W_W, b64);
  if (!bh || !xe || !r || !w) return QXD_ENOMEM;
  double nb;
  QXD_TRY(norm_full(h, (const double2*)b, &nb, s));
  QXD_TRY(qxd_eo_source(h, bh, b, s));
  QXD_HIP(hipMemcpyAsync(r, bh, b64, hipMemcpyDeviceToDevice, s));
  // snapshots (x_k, r_k) at every `stride`-th restart; when more than `cap` are
  // held, every other one is dropped and the stride doubles, so at most cap
  // snapshots, evenly spread over the solve, are kept
  std::vector<double2*> snaps;
  const int cap = 2 * npairs + 2;
  int64_t cycle = 0, stride = 1;
  qxd_status cb_status = QXD_OK;
  // pairs are recorded while |r_k| > 1e-6 |bhat|: e_k = x* - x_k solves
  // D_hat e_k = r_k - r*, with |r*| <= 1e-10 |b|, so later pairs would carry a
  // relative error above 1e-4
  blas_norm2<double2>(h, bh, n64, h->scal + S_BH, s);
  QXD_TRY(read_scal(h, S_BH, 1, s));
  const double rec_floor = 1e-6 * std::sqrt(h->scal_host[S_BH]);
  std::function<qxd_status()> on_cycle = [&]() -> qxd_status {
    if (std::sqrt(h->scal_host[S_FRR]) < rec_floor) return QXD_OK;
    if (cycle++ % stride != 0) return QXD_OK;
    double2 *xs = nullptr, *rs = nullptr;
    if (!dev_alloc(&xs, b64) || !dev_alloc(&rs, b64)) {
      if (xs) (void)hipFree(xs);
      cb_status = QXD_ENOMEM;
      return QXD_ENOMEM;
    }
    QXD_HIP(hipMemcpyAsync(xs, xe, b64, hipMemcpyDeviceToDevice, s));
    QXD_HIP(hipMemcpyAsync(rs, r, b64, hipMemcpyDeviceToDevice, s));
    snaps.push_back(xs);
    snaps.push_back(rs);
    if ((int)snaps.size() / 2 > cap) {
      QXD_HIP(hipStreamSynchronize(s));
      std::vector<double2*> keep;
      for (size_t k = 0; k < snaps.size() / 2; ++k) {
        if (k % 2 == 0) {
          keep.push_back(snaps[2 * k]);
          keep.push_back(snaps[2 * k + 1]);
        } else {
          (void)hipFree(snaps[2 * k]);
          (void)hipFree(snaps[2 * k + 1]);
        }
      }
      snaps.swap(keep);
      stride *= 2;
    }
    return QXD_OK;
  };
  FgcrResult fr;
  InnerOp op{0};
  qxd_status rc = fgcr<double2>(h, op, Precond{}, 1 << 30, xe, r, n64, 4, 1e-10 * nb, 50000, &fr, s, &on_cycle);
  int nsnap = (int)snaps.size() / 2;
  if (rc == QXD_OK && nsnap > 0) {
    int take = std::min(npairs, nsnap);
    h->scal_host[S_ONE] = 1.0;
    QXD_HIP(hipMemcpyAsync(h->scal + S_ONE, h->scal_host + S_ONE, sizeof(double), hipMemcpyHostToDevice, s));
    size_t half32 = (size_t)6 * h->Ve;
    for (int i = 0; i < take; ++i) {
      int k = take == 1 ? nsnap - 1 : (int)((int64_t)i * (nsnap - 1) / (take - 1));
      blas_sub_norm<double2>(h, w, xe, snaps[2 * k], n64, h->scal + S_RT, s);  // e_k = x* - x_k
      blas_down(h, (float4*)e_out + i * half32, w, S_ONE, s);
      blas_down(h, (float4*)r_out + i * half32, snaps[2 * k + 1], S_ONE, s);
    }
    QXD_HIP(hipStreamSynchronize(s));
    if (n_harvested) *n_harvested = take;
  } else if (n_harvested) {
    *n_harvested = 0;
  }
  QXD_HIP(hipStreamSynchronize(s));
  for (double2* p : snaps) (void)hipFree(p);
  if (cb_status != QXD_OK) return cb_status;
  return rc;
}
