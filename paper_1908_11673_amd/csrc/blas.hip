// BLAS-1 kernels and deterministic reductions for the Krylov solvers.
//
// Vectors are half fields viewed as flat arrays of 16-byte words: double2 (one
// complex128) or float4 (two complex64).  Reductions are two-pass: each of a
// fixed number of workgroups reduces its grid-stride share (wave64 shuffles,
// then LDS) into one partial, and a single-workgroup kernel sums the partials in
// a fixed order, so results are bitwise reproducible run to run.  Scalars such as
// CG's alpha and beta are read by the update kernels straight from device
// memory; the host never waits inside an iteration.
#include "blas.hpp"

__device__ inline double red_block(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

// ---- word helpers ---------------------------------------------------------

__device__ inline double wnorm2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double wnorm2(float4 a) { return (double)(a.x * a.x + a.y * a.y) + (double)(a.z * a.z + a.w * a.w); }
// conj(a) b
__device__ inline void wcdot(double2 a, double2 b, double& re, double& im) {
  re += a.x * b.x + a.y * b.y;
  im += a.x * b.y - a.y * b.x;
}
__device__ inline void wcdot(float4 a, float4 b, double& re, double& im) {
  re += (double)(a.x * b.x + a.y * b.y) + (double)(a.z * b.z + a.w * b.w);
  im += (double)(a.x * b.y - a.y * b.x) + (double)(a.z * b.w - a.w * b.z);
}
// y + (cr + i ci) x
__device__ inline double2 wcaxpy(double2 y, double cr, double ci, double2 x) {
  return make_double2(y.x + cr * x.x - ci * x.y, y.y + cr * x.y + ci * x.x);
}
__device__ inline float4 wcaxpy(float4 y, double crd, double cid, float4 x) {
  float cr = (float)crd, ci = (float)cid;
  return make_float4(y.x + cr * x.x - ci * x.y, y.y + cr * x.y + ci * x.x, y.z + cr * x.z - ci * x.w,
                     y.w + cr * x.w + ci * x.z);
}
__device__ inline double2 wscale(double2 x, double s) { return make_double2(s * x.x, s * x.y); }
__device__ inline float4 wscale(float4 x, double sd) {
  float s = (float)sd;
  return make_float4(s * x.x, s * x.y, s * x.z, s * x.w);
}
__device__ inline double2 wadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline float4 wadd(float4 a, float4 b) { return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w); }
__device__ inline double2 wsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline float4 wsub(float4 a, float4 b) { return make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w); }
__device__ inline bool wfinite(double2 a) { return isfinite(a.x) && isfinite(a.y); }

// Solver vectors are streamed once per kernel: loads and stores carry the
// non-temporal hint (ld_stream, st_stream).
#define GRID_STRIDE(i, n) for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (size_t)gridDim.x * blockDim.x)

// Traversal in rounds with QXD_UNR elements in flight per thread: in a round
// workgroup b takes the QXD_UNR * blockDim contiguous elements that start at
// round_start + b QXD_UNR blockDim, thread t the elements t, t + blockDim, ...
// of them, and all loads of the round (load(i) returns an element's words) are
// issued before the first element is used (use(i, words)).  The elements after
// the last full round go one at a time in a plain grid-stride loop.  (With a
// plain grid-stride loop, even unrolled, the compiler waits for an element's
// loads before issuing the next element's; with the elements of a round a grid
// apart, each wave reads several distant regions at once, which measured
// slower than contiguous rounds.)  The order is fixed, so the reductions stay
// reproducible.
#define QXD_UNR 4
template <class Load, class Use>
__device__ __forceinline__ void stream_for(size_t n, Load load, Use use) {
  const size_t B = blockDim.x, span = (size_t)gridDim.x * QXD_UNR * B;  // elements per round
  size_t start = 0;
  for (; start + span <= n; start += span) {
    const size_t i0 = start + (size_t)blockIdx.x * QXD_UNR * B + threadIdx.x;
    decltype(load(i0)) w[QXD_UNR];
#pragma unroll
    for (int u = 0; u < QXD_UNR; ++u) w[u] = load(i0 + u * B);
#pragma unroll
    for (int u = 0; u < QXD_UNR; ++u) use(i0 + u * B, w[u]);
  }
  for (size_t i = start + (size_t)blockIdx.x * B + threadIdx.x; i < n; i += (size_t)gridDim.x * B) use(i, load(i));
}
template <class VT>
struct W2 {
  VT a, b;
};

// ---- kernels ---------------------------------------------------------------

__global__ __launch_bounds__(QXD_BLOCK) void k_final_sum(const double* __restrict__ partial, int n, int nvals,
                                                         int stride, double* __restrict__ out) {
  __shared__ double sh[QXD_BLOCK / 64];
  for (int v = 0; v < nvals; ++v) {
    double a = 0.0;
    for (int i = threadIdx.x; i < n; i += QXD_BLOCK) a += partial[(size_t)v * stride + i];
    double s = red_block(a, sh);
    if (threadIdx.x == 0) out[v] = s;
  }
}

template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_norm2(const VT* __restrict__ x, size_t n, double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double a = 0.0;
  stream_for(n, [&](size_t i) { return ld_stream(&x[i]); }, [&](size_t, VT v) { a += wnorm2(v); });
  double s = red_block(a, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_cdot(const VT* __restrict__ x, const VT* __restrict__ y, size_t n,
                                                    double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double re = 0.0, im = 0.0;
  stream_for(n, [&](size_t i) { return W2<VT>{ld_stream(&x[i]), ld_stream(&y[i])}; },
             [&](size_t, W2<VT> v) { wcdot(v.a, v.b, re, im); });
  double s = red_block(re, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  s = red_block(im, sh);
  if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s;
}

// CG: alpha = zz / ww; x += alpha p; r -= alpha w; partial |r|^2
template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_cg_xr(VT* __restrict__ x, VT* __restrict__ r, const VT* __restrict__ p,
                                                     const VT* __restrict__ w, size_t n, const double* __restrict__ scal,
                                                     int i_zz, int i_ww, double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double alpha = scal[i_zz] / scal[i_ww];
  double a = 0.0;
  struct W4 {
    VT x, p, r, w;
  };
  stream_for(
      n, [&](size_t i) { return W4{ld_stream(&x[i]), ld_stream(&p[i]), ld_stream(&r[i]), ld_stream(&w[i])}; },
      [&](size_t i, W4 v) {
        st_stream(&x[i], wcaxpy(v.x, alpha, 0.0, v.p));
        VT rr = wcaxpy(v.r, -alpha, 0.0, v.w);
        st_stream(&r[i], rr);
        a += wnorm2(rr);
      });
  double s = red_block(a, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// CG: beta = zz_new / zz_old; p = z + beta p
template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_cg_p(VT* __restrict__ p, const VT* __restrict__ z, size_t n,
                                                    const double* __restrict__ scal, int i_new, int i_old) {
  double beta = scal[i_new] / scal[i_old];
  stream_for(n, [&](size_t i) { return W2<VT>{ld_stream(&z[i]), ld_stream(&p[i])}; },
             [&](size_t i, W2<VT> v) { st_stream(&p[i], wcaxpy(v.a, beta, 0.0, v.b)); });
}

// r = b - w; partial |r|^2
template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_sub_norm(VT* __restrict__ r, const VT* __restrict__ b,
                                                        const VT* __restrict__ w, size_t n,
                                                        double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double a = 0.0;
  stream_for(n, [&](size_t i) { return W2<VT>{ld_stream(&b[i]), ld_stream(&w[i])}; },
             [&](size_t i, W2<VT> bw) {
               VT v = wsub(bw.a, bw.b);
               if (r) st_stream(&r[i], v);  // r = nullptr: the norm only
               a += wnorm2(v);
             });
  double s = red_block(a, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// The multi-vector kernels below are instantiated for every basis size K (0 ..
// QXD_MAXKV): with the count fixed at compile time all loads of an element
// (in groups of QXD_KGROUP) are issued before the first one is used, where a
// run-time count left the compiler waiting for each load in turn.  The
// arithmetic and its order are those of a plain loop over j.
#define QXD_KGROUP 16

// dots (basis_j, v) for j < K: partial[(2j) G + b] = Re, [(2j+1) G + b] = Im
template <class VT, int K>
__global__ __launch_bounds__(QXD_BLOCK) void k_mdot(Ptrs basis, const VT* __restrict__ v, size_t n,
                                                    double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double re[K > 0 ? K : 1], im[K > 0 ? K : 1];
#pragma unroll
  for (int j = 0; j < K; ++j) re[j] = im[j] = 0.0;
  GRID_STRIDE(i, n) {
    VT vi = ld_stream(&v[i]);
#pragma unroll
    for (int j0 = 0; j0 < K; j0 += QXD_KGROUP) {
      VT bj[QXD_KGROUP];
#pragma unroll
      for (int j = 0; j < QXD_KGROUP; ++j)
        if (j0 + j < K) bj[j] = ld_stream(&((const VT*)basis.p[j0 + j])[i]);
#pragma unroll
      for (int j = 0; j < QXD_KGROUP; ++j)
        if (j0 + j < K) wcdot(bj[j], vi, re[j0 + j], im[j0 + j]);
    }
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double s = red_block(re[j], sh);
    if (threadIdx.x == 0) partial[(size_t)(2 * j) * gridDim.x + blockIdx.x] = s;
    s = red_block(im[j], sh);
    if (threadIdx.x == 0) partial[(size_t)(2 * j + 1) * gridDim.x + blockIdx.x] = s;
  }
}

// v -= sum_{j < K} c_j basis_j (c complex at coef[2j], coef[2j+1]); partial |v|^2
template <class VT, int K>
__global__ __launch_bounds__(QXD_BLOCK) void k_mupdate(VT* __restrict__ v, Ptrs basis,
                                                       const double* __restrict__ coef, size_t n,
                                                       double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  double a = 0.0;
  GRID_STRIDE(i, n) {
    VT vi = ld_stream(&v[i]);
#pragma unroll
    for (int j0 = 0; j0 < K; j0 += QXD_KGROUP) {
      VT bj[QXD_KGROUP];
#pragma unroll
      for (int j = 0; j < QXD_KGROUP; ++j)
        if (j0 + j < K) bj[j] = ld_stream(&((const VT*)basis.p[j0 + j])[i]);
#pragma unroll
      for (int j = 0; j < QXD_KGROUP; ++j)
        if (j0 + j < K) vi = wcaxpy(vi, -coef[2 * (j0 + j)], -coef[2 * (j0 + j) + 1], bj[j]);
    }
    st_stream(&v[i], vi);
    a += wnorm2(vi);
  }
  double s = red_block(a, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// v *= 1/sqrt(scal[i_n2]); partial (v, r).  A norm that is zero or not finite
// (a Krylov breakdown, e.g. on a vanishing source) sets v = 0 instead, so that
// the update that follows leaves the residual unchanged.
template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_scale_cdot(VT* __restrict__ v, const VT* __restrict__ r, size_t n,
                                                          const double* __restrict__ scal, int i_n2,
                                                          double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  const double n2 = scal[i_n2];
  const bool ok = n2 > 0.0 && n2 < INFINITY;
  const double sc = ok ? 1.0 / sqrt(n2) : 0.0;
  double re = 0.0, im = 0.0;
  stream_for(n, [&](size_t i) { return W2<VT>{ld_stream(&v[i]), ld_stream(&r[i])}; },
             [&](size_t i, W2<VT> w) {
               VT vi = ok ? wscale(w.a, sc) : VT{};
               st_stream(&v[i], vi);
               wcdot(vi, w.b, re, im);
             });
  double s = red_block(re, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
  s = red_block(im, sh);
  if (threadIdx.x == 0) partial[gridDim.x + blockIdx.x] = s;
}

// r -= c v (c complex at scal[i_c]), also written to r_copy unless that is
// null; partial |r|^2
template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_r_update(VT* __restrict__ r, const VT* __restrict__ v, size_t n,
                                                        const double* __restrict__ scal, int i_c,
                                                        double* __restrict__ partial, VT* __restrict__ r_copy) {
  __shared__ double sh[QXD_BLOCK / 64];
  double cr = scal[i_c], ci = scal[i_c + 1];
  double a = 0.0;
  stream_for(n, [&](size_t i) { return W2<VT>{ld_stream(&r[i]), ld_stream(&v[i])}; },
             [&](size_t i, W2<VT> w) {
               VT ri = wcaxpy(w.a, -cr, -ci, w.b);
               st_stream(&r[i], ri);
               if (r_copy) st_stream(&r_copy[i], ri);
               a += wnorm2(ri);
             });
  double s = red_block(a, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

// x += sum_{j < K} c_j basis_j
template <class VT, int K>
__global__ __launch_bounds__(QXD_BLOCK) void k_multi_axpy(VT* __restrict__ x, Ptrs basis,
                                                          const double* __restrict__ coef, size_t n) {
  GRID_STRIDE(i, n) {
    VT xi = ld_stream(&x[i]);
#pragma unroll
    for (int j0 = 0; j0 < K; j0 += QXD_KGROUP) {
      VT bj[QXD_KGROUP];
#pragma unroll
      for (int j = 0; j < QXD_KGROUP; ++j)
        if (j0 + j < K) bj[j] = ld_stream(&((const VT*)basis.p[j0 + j])[i]);
#pragma unroll
      for (int j = 0; j < QXD_KGROUP; ++j)
        if (j0 + j < K) xi = wcaxpy(xi, coef[2 * (j0 + j)], coef[2 * (j0 + j) + 1], bj[j]);
    }
    st_stream(&x[i], xi);
  }
}

template <class VT>
__global__ __launch_bounds__(QXD_BLOCK) void k_zero(VT* __restrict__ x, size_t n) {
  GRID_STRIDE(i, n) x[i] = VT{};
}

// FP64 half field [12][Ve] double2 -> FP32 half field [6][Ve] float4: word
// j Ve + h holds components 2j and 2j+1 of site h.
// d = s / sqrt(scal[i_n2])
__global__ __launch_bounds__(QXD_BLOCK) void k_down(float4* __restrict__ d, const double2* __restrict__ s, size_t Ve,
                                                    const double* __restrict__ scal, int i_n2) {
  double sc = 1.0 / sqrt(scal[i_n2]);
  stream_for(
      6 * Ve,
      [&](size_t i) {
        size_t j = i / Ve, h = i - j * Ve;
        return W2<double2>{s[(2 * j) * Ve + h], s[(2 * j + 1) * Ve + h]};
      },
      [&](size_t i, W2<double2> w) {
        d[i] = make_float4((float)(sc * w.a.x), (float)(sc * w.a.y), (float)(sc * w.b.x), (float)(sc * w.b.y));
      });
}

// x (FP64) += sqrt(scal[i]) e (FP32), same component map as k_down
__global__ __launch_bounds__(QXD_BLOCK) void k_up_acc(double2* __restrict__ x, const float4* __restrict__ e, size_t Ve,
                                                      const double* __restrict__ scal, int i_n2) {
  double sc = sqrt(scal[i_n2]);
  // the elements of a round touch distinct words of x, so their loads may all
  // precede the stores
  struct W3 {
    float4 v;
    double2 a, b;
  };
  stream_for(
      6 * Ve,
      [&](size_t i) {
        size_t j = i / Ve, h = i - j * Ve;
        return W3{e[i], x[(2 * j) * Ve + h], x[(2 * j + 1) * Ve + h]};
      },
      [&](size_t i, W3 w) {
        size_t j = i / Ve, h = i - j * Ve;
        x[(2 * j) * Ve + h] = make_double2(w.a.x + sc * (double)w.v.x, w.a.y + sc * (double)w.v.y);
        x[(2 * j + 1) * Ve + h] = make_double2(w.b.x + sc * (double)w.v.z, w.b.y + sc * (double)w.v.w);
      });
}

// ---- host launchers -------------------------------------------------------

void launch_final_sum(const double* partial, int n, int nvals, int stride, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(QXD_BLOCK), 0, s, partial, n, nvals, stride, out);
}

template <class VT>
void blas_norm2(qxd_handle* h, const VT* x, size_t n, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(k_norm2<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, x, n, h->partial);
  launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, slot, s);
}
template <class VT>
void blas_cdot(qxd_handle* h, const VT* x, const VT* y, size_t n, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(k_cdot<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, x, y, n, h->partial);
  launch_final_sum(h->partial, QXD_NRED, 2, QXD_NRED, slot, s);
}
template <class VT>
void blas_cg_xr(qxd_handle* h, VT* x, VT* r, const VT* p, const VT* w, size_t n, int i_zz, int i_ww, int i_rr,
                hipStream_t s) {
  hipLaunchKernelGGL(k_cg_xr<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, x, r, p, w, n, h->scal, i_zz, i_ww,
                     h->partial);
  launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, h->scal + i_rr, s);
}
template <class VT>
void blas_cg_p(qxd_handle* h, VT* p, const VT* z, size_t n, int i_new, int i_old, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_p<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, p, z, n, h->scal, i_new, i_old);
}
template <class VT>
void blas_sub_norm(qxd_handle* h, VT* r, const VT* b, const VT* w, size_t n, double* slot, hipStream_t s) {
  hipLaunchKernelGGL(k_sub_norm<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, r, b, w, n, h->partial);
  launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, slot, s);
}
// one case per basis size 0 .. QXD_MAXKV
#define QXD_K_CASES(X)                                                                                         \
  X(0) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12) X(13) X(14) X(15) X(16) X(17) X(18) X(19) \
  X(20) X(21) X(22) X(23) X(24) X(25) X(26) X(27) X(28) X(29) X(30) X(31) X(32)
static_assert(QXD_MAXKV == 32, "QXD_K_CASES lists the basis sizes 0 .. QXD_MAXKV");

template <class VT>
void blas_mdot(qxd_handle* h, const Ptrs& basis, int k, const VT* v, size_t n, double* slots, hipStream_t s) {
  if (k == 0) return;  // no dots
  switch (k) {
#define QXD_CASE(K)                                                                                             \
  case K:                                                                                                     \
    hipLaunchKernelGGL((k_mdot<VT, K>), dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, basis, v, n, h->partial);      \
    break;
    QXD_K_CASES(QXD_CASE)
#undef QXD_CASE
    default: return;  // callers keep 0 <= k <= QXD_MAXKV
  }
  launch_final_sum(h->partial, QXD_NRED, 2 * k, QXD_NRED, slots, s);
}
template <class VT>
void blas_mupdate(qxd_handle* h, VT* v, const Ptrs& basis, int k, const double* coef, size_t n, double* slot,
                  hipStream_t s) {
  switch (k) {
#define QXD_CASE(K)                                                                                             \
  case K:                                                                                                     \
    hipLaunchKernelGGL((k_mupdate<VT, K>), dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, v, basis, coef, n,           \
                       h->partial);                                                                           \
    break;
    QXD_K_CASES(QXD_CASE)
#undef QXD_CASE
    default: return;
  }
  launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, slot, s);
}
template <class VT>
void blas_scale_cdot(qxd_handle* h, VT* v, const VT* r, size_t n, int i_n2, double* slots, hipStream_t s) {
  hipLaunchKernelGGL(k_scale_cdot<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, v, r, n, h->scal, i_n2, h->partial);
  launch_final_sum(h->partial, QXD_NRED, 2, QXD_NRED, slots, s);
}
template <class VT>
void blas_r_update(qxd_handle* h, VT* r, const VT* v, size_t n, int i_c, double* slot, hipStream_t s, VT* r_copy) {
  hipLaunchKernelGGL(k_r_update<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, r, v, n, h->scal, i_c, h->partial,
                     r_copy);
  launch_final_sum(h->partial, QXD_NRED, 1, QXD_NRED, slot, s);
}
template <class VT>
void blas_multi_axpy(qxd_handle* h, VT* x, const Ptrs& basis, int k, const double* coef, size_t n, hipStream_t s) {
  if (k == 0) return;  // x unchanged
  switch (k) {
#define QXD_CASE(K)                                                                                             \
  case K:                                                                                                     \
    hipLaunchKernelGGL((k_multi_axpy<VT, K>), dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, x, basis, coef, n);      \
    break;
    QXD_K_CASES(QXD_CASE)
#undef QXD_CASE
    default: return;
  }
}
template <class VT>
void blas_zero(VT* x, size_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_zero<VT>, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, x, n);
}
void blas_down(qxd_handle* h, float4* d, const double2* src, int i_n2, hipStream_t s) {
  hipLaunchKernelGGL(k_down, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, d, src, (size_t)h->Ve, h->scal, i_n2);
}
void blas_up_acc(qxd_handle* h, double2* x, const float4* e, int i_n2, hipStream_t s) {
  hipLaunchKernelGGL(k_up_acc, dim3(QXD_NRED), dim3(QXD_BLOCK), 0, s, x, e, (size_t)h->Ve, h->scal, i_n2);
}

#define INST(VT)                                                                                        \
  template void blas_norm2<VT>(qxd_handle*, const VT*, size_t, double*, hipStream_t);                  \
  template void blas_cdot<VT>(qxd_handle*, const VT*, const VT*, size_t, double*, hipStream_t);        \
  template void blas_cg_xr<VT>(qxd_handle*, VT*, VT*, const VT*, const VT*, size_t, int, int, int,      \
                               hipStream_t);                                                            \
  template void blas_cg_p<VT>(qxd_handle*, VT*, const VT*, size_t, int, int, hipStream_t);              \
  template void blas_sub_norm<VT>(qxd_handle*, VT*, const VT*, const VT*, size_t, double*, hipStream_t); \
  template void blas_mdot<VT>(qxd_handle*, const Ptrs&, int, const VT*, size_t, double*, hipStream_t);  \
  template void blas_mupdate<VT>(qxd_handle*, VT*, const Ptrs&, int, const double*, size_t, double*,    \
                                 hipStream_t);                                                          \
  template void blas_scale_cdot<VT>(qxd_handle*, VT*, const VT*, size_t, int, double*, hipStream_t);    \
  template void blas_r_update<VT>(qxd_handle*, VT*, const VT*, size_t, int, double*, hipStream_t, VT*); \
  template void blas_multi_axpy<VT>(qxd_handle*, VT*, const Ptrs&, int, const double*, size_t,          \
                                    hipStream_t);                                                       \
  template void blas_zero<VT>(VT*, size_t, hipStream_t);

INST(double2)
INST(float4)
