// BLAS-1 launchers for the solvers (see blas.hip).
#pragma once

#include "qxd_internal.hpp"

#define QXD_NRED 1024   // workgroups of a reduction kernel (fixed: results are reproducible)
#define QXD_MAXKV 32    // largest Krylov basis the fused multi-dot kernels take

struct Ptrs {
  const void* p[QXD_MAXKV];
};

template <class VT> void blas_norm2(qxd_handle* h, const VT* x, size_t n, double* slot, hipStream_t s);
template <class VT> void blas_cdot(qxd_handle* h, const VT* x, const VT* y, size_t n, double* slot, hipStream_t s);
template <class VT>
void blas_cg_xr(qxd_handle* h, VT* x, VT* r, const VT* p, const VT* w, size_t n, int i_zz, int i_ww, int i_rr,
                hipStream_t s);
template <class VT> void blas_cg_p(qxd_handle* h, VT* p, const VT* z, size_t n, int i_new, int i_old, hipStream_t s);
template <class VT>
void blas_sub_norm(qxd_handle* h, VT* r, const VT* b, const VT* w, size_t n, double* slot, hipStream_t s);
template <class VT>
void blas_mdot(qxd_handle* h, const Ptrs& basis, int k, const VT* v, size_t n, double* slots, hipStream_t s);
template <class VT>
void blas_mupdate(qxd_handle* h, VT* v, const Ptrs& basis, int k, const double* coef, size_t n, double* slot,
                  hipStream_t s);
template <class VT>
void blas_scale_cdot(qxd_handle* h, VT* v, const VT* r, size_t n, int i_n2, double* slots, hipStream_t s);
// r -= c v; with r_copy the new r is written there too
template <class VT>
void blas_r_update(qxd_handle* h, VT* r, const VT* v, size_t n, int i_c, double* slot, hipStream_t s,
                   VT* r_copy = nullptr);
template <class VT>
void blas_multi_axpy(qxd_handle* h, VT* x, const Ptrs& basis, int k, const double* coef, size_t n, hipStream_t s);
template <class VT> void blas_zero(VT* x, size_t n, hipStream_t s);
// FP64 half field <-> FP32 half field (the layouts interleave components differently)
void blas_down(qxd_handle* h, float4* d, const double2* src, int i_n2, hipStream_t s);
void blas_up_acc(qxd_handle* h, double2* x, const float4* e, int i_n2, hipStream_t s);
