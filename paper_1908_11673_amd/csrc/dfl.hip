// Inexact deflation for SAP-preconditioned GCR (Sec. 4.4, DFL+SAP+GCR), FP32.
//
// A deflation subspace is spanned by ns vectors made rich in low modes of D by
// approximate inverse iteration (v <- M_sap v, normalised, nit times), then cut
// into the 4^4 SAP blocks and orthonormalised block by block: W maps a coarse
// vector c = (c_{B,k}) to sum_{B,k} c_{B,k} w_{B,k}.  The little operator
// A = W^+ D W couples a block to itself and its eight face neighbours only and
// is stored as 9 dense ns x ns blocks per block row.  The preconditioner is the
// two-level one of inexact deflation: c from nc GCR steps on A c = W^+ eta
// (the coarse system is solved only approximately), psi = W c, then
// psi + M_sap (eta - D psi).  The subspace belongs to the operator it was made
// with: one subspace per quark charge; qxd_dfl_little rebuilds A for another
// operator from the same W.
//
// Layout: W in block order (blocks colour-major as for SAP, plain slots), basis
// vectors of a block contiguous: [B][k][6 float4 components][256 slots].  A is
// [B][n][k][l] complex float (column k of the ns x ns block contiguous, so the
// threads of the rows l of one block read consecutive words), n = 0 the block
// itself, 1 + 2 mu its +mu neighbour, 2 + 2 mu its -mu neighbour; nbr[B][n]
// names those blocks.  Coarse
// vectors are [B][k] complex float.  One workgroup per block (one thread per
// site) orthonormalises, builds A (the in-block part of D through the same LDS
// exchange as SAP, the face hops by the face threads), restricts and prolongs.
#include <algorithm>
#include <cmath>
#include <new>

#include "blas.hpp"
#include "sap_blocks.hpp"

struct qxd_dfl {
  int ns = 0, nblk = 0;
  SapGeo sb{};
  Geo geo{};              // the lattice it was made for
  const qxd_handle* op = nullptr;  // the handle whose operator A was built for
  uint64_t gen = 0;       // that handle's setup_gen then (0: none)
  bool has_basis = false;
  float4* W = nullptr;    // [B][ns][6][256]
  float2* A = nullptr;    // [B][9][ns (k)][ns (l)]
  int* nbr = nullptr;     // [B][9]
  float2 *cb = nullptr, *cx = nullptr, *cr = nullptr;  // coarse source, solution, residual
  float2 *cz = nullptr, *cw = nullptr;                 // QXD_DFL_MAXNC coarse directions and their images
  float4 *psi = nullptr, *t = nullptr, *xs = nullptr;  // FP32 full, full and even half fields
};

namespace {

constexpr int kDflMaxNs = QXD_DFL_MAXNS;
constexpr int kDflMaxNc = QXD_DFL_MAXNC;

// device scalar slots (after the multi-shift solver's)
enum { S_DC = 3880, S_DN = S_DC + 2 * kDflMaxNc, S_DA = S_DN + 2, S_DX = S_DA + 2, S_DY = S_DX + 2, S_DEND = S_DY + 2 };
static_assert(S_DEND <= QXD_NSCAL - 8, "scalar slots");

__device__ __forceinline__ void dfl_site(const Geo& g, const SapGeo& sb, int B, int t, int& x0, int& x1, int& x2,
                                         int& x3, int& p, size_t& h) {
  const int colour = B >= sb.nhalf ? 1 : 0;
  int c0, c1, c2, c3, l0, l1, l2, l3;
  sap_block_coords(sb, colour, B - colour * sb.nhalf, c0, c1, c2, c3);
  sap_local<false>(t, l0, l1, l2, l3);
  x0 = kSapB * c0 + l0;
  x1 = kSapB * c1 + l1;
  x2 = kSapB * c2 + l2;
  x3 = kSapB * c3 + l3;
  p = (x0 + x1 + x2 + x3) & 1;
  h = geo_half(g, x0, x1, x2, x3);
}

template <int MU>
__device__ __forceinline__ void dfl_nb(const Geo& g, const SapGeo& sb, int x0, int x1, int x2, int x3, int* out) {
  bool neg;
  int y0 = x0 + (MU == 0 ? kSapB - 1 : 0), y1 = x1 + (MU == 1 ? kSapB - 1 : 0), y2 = x2 + (MU == 2 ? kSapB - 1 : 0),
      y3 = x3 + (MU == 3 ? kSapB - 1 : 0);
  geo_step<MU, +1>(g, y0, y1, y2, y3, neg);
  out[0] = sap_bsite<false>(sb, y0, y1, y2, y3) / kSapSites;
  y0 = x0, y1 = x1, y2 = x2, y3 = x3;
  geo_step<MU, -1>(g, y0, y1, y2, y3, neg);
  out[1] = sap_bsite<false>(sb, y0, y1, y2, y3) / kSapSites;
}

// The neighbour table: from each block's origin (and its far corner along mu).
__global__ void k_dfl_nbr(Geo g, SapGeo sb, int nblk, int* __restrict__ nbr) {
  const int B = blockIdx.x * blockDim.x + threadIdx.x;
  if (B >= nblk) return;
  const int colour = B >= sb.nhalf ? 1 : 0;
  int c0, c1, c2, c3;
  sap_block_coords(sb, colour, B - colour * sb.nhalf, c0, c1, c2, c3);
  const int x0 = kSapB * c0, x1 = kSapB * c1, x2 = kSapB * c2, x3 = kSapB * c3;
  int* o = nbr + (size_t)9 * B;
  o[0] = B;
  dfl_nb<0>(g, sb, x0, x1, x2, x3, o + 1);
  dfl_nb<1>(g, sb, x0, x1, x2, x3, o + 3);
  dfl_nb<2>(g, sb, x0, x1, x2, x3, o + 5);
  dfl_nb<3>(g, sb, x0, x1, x2, x3, o + 7);
}

// A site's 12 components of a basis vector (block order, stride kSapSites),
// loaded with the non-temporal hint: the basis is streamed once per use.
__device__ __forceinline__ void dfl_wload(const float4* w, cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    const float4 v = ld_stream(w + (size_t)j * kSapSites);
    s[2 * j] = mk(v.x, v.y);
    s[2 * j + 1] = mk(v.z, v.w);
  }
}

__device__ __forceinline__ double dfl_wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// conj(a) . b over a site's 12 components
__device__ __forceinline__ void dfl_cdot(const cx<float> a[12], const cx<float> b[12], double& re, double& im) {
  float r = 0.f, i = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    r += a[c].re * b[c].re + a[c].im * b[c].im;
    i += a[c].re * b[c].im - a[c].im * b[c].re;
  }
  re = r;
  im = i;
}

// Block orthonormalisation of the ns vectors v (FP32 full fields, `full` float4
// apart): classical Gram-Schmidt applied twice per vector (the restrictions of
// smooth vectors to a block are nearly parallel), dots summed in FP64.
__global__ __launch_bounds__(kSapSites) void k_dfl_orth(Geo g, SapGeo sb, int ns, const float4* __restrict__ v,
                                                        size_t full, float4* __restrict__ W) {
  __shared__ double red[kSapSites / 64][2 * kDflMaxNs];
  __shared__ double tot[2 * kDflMaxNs];
  const int B = blockIdx.x, t = threadIdx.x, wave = t >> 6, lane = t & 63;
  int x0, x1, x2, x3, p;
  size_t h;
  dfl_site(g, sb, B, t, x0, x1, x2, x3, p, h);
  const size_t Ve = g.Ve;
  float4* wb = W + (size_t)B * ns * 6 * kSapSites;
  for (int k = 0; k < ns; ++k) {
    cx<float> x[12];
    sp_load(v + k * full + (size_t)p * 6 * Ve, Ve, h, x);
    for (int pass = 0; pass < 2 && k > 0; ++pass) {
      for (int j = 0; j < k; ++j) {
        cx<float> wj[12];
        sp_load(wb + (size_t)j * 6 * kSapSites, kSapSites, t, wj);
        double re, im;
        dfl_cdot(wj, x, re, im);
        re = dfl_wave_sum(re);
        im = dfl_wave_sum(im);
        if (lane == 0) {
          red[wave][2 * j] = re;
          red[wave][2 * j + 1] = im;
        }
      }
      __syncthreads();
      if (t < 2 * k) tot[t] = red[0][t] + red[1][t] + red[2][t] + red[3][t];
      __syncthreads();
      for (int j = 0; j < k; ++j) {
        cx<float> wj[12];
        sp_load(wb + (size_t)j * 6 * kSapSites, kSapSites, t, wj);
        const cx<float> d = mk((float)tot[2 * j], (float)tot[2 * j + 1]);
#pragma unroll
        for (int c = 0; c < 12; ++c) x[c] = x[c] - d * wj[c];
      }
      __syncthreads();
    }
    double n2 = 0.0;
#pragma unroll
    for (int c = 0; c < 12; ++c) n2 += (double)norm2(x[c]);
    n2 = dfl_wave_sum(n2);
    if (lane == 0) red[wave][0] = n2;
    __syncthreads();
    n2 = red[0][0] + red[1][0] + red[2][0] + red[3][0];
    __syncthreads();
    const float sc = n2 > 0.0 ? (float)(1.0 / sqrt(n2)) : 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) x[c] = sc * x[c];
    sp_store(wb + (size_t)k * 6 * kSapSites, kSapSites, t, x);
  }
}

// dst[l * stride] = sum over the block of conj(w_l) . f, for l < ns; wl points
// at the thread's slot of its block's first basis vector (null: contributes 0).
// STREAM: the basis is read once (restriction), else it is read again by the
// same workgroup (little operator) and stays cacheable.
template <bool STREAM>
__device__ __forceinline__ void dfl_project(float2 (*red)[kDflMaxNs], const float4* wl, const cx<float> f[12],
                                            int ns, float2* __restrict__ dst, size_t stride) {
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  for (int l = 0; l < ns; ++l) {
    double re = 0.0, im = 0.0;
    if (wl) {
      cx<float> w[12];
      if (STREAM)
        dfl_wload(wl + (size_t)l * 6 * kSapSites, w);
      else
        sp_load(wl + (size_t)l * 6 * kSapSites, kSapSites, 0, w);
      dfl_cdot(w, f, re, im);
    }
    re = dfl_wave_sum(re);
    im = dfl_wave_sum(im);
    if (lane == 0) red[wave][l] = make_float2((float)re, (float)im);
  }
  __syncthreads();
  if (t < ns) {
    float2 a = red[0][t], b = red[1][t], c = red[2][t], d = red[3][t];
    dst[t * stride] = make_float2(a.x + b.x + c.x + d.x, a.y + b.y + c.y + d.y);
  }
  __syncthreads();
}

// The two face hops of w along MU that leave block B, projected on the
// neighbours' bases: into A[B'][n'][.][k] of the neighbour row blocks.
template <int MU>
__device__ __forceinline__ void dfl_faces(const Geo& g, const SapGeo& sb, float2 (*red)[kDflMaxNs], int B, int x0,
                                          int x1, int x2, int x3, int l, const cx<float> w[12], const cx<float> u[9],
                                          const float4* __restrict__ W, const float2* __restrict__ Vb,
                                          const int* __restrict__ nbr, int ns, int k, float2* __restrict__ A) {
  const size_t bsz = (size_t)ns * 6 * kSapSites;
  {  // +MU: y = x + MU in B' = B + MU gets -(1/2) (1 + g_MU) U(x, MU)^+ w(x)
    const int Bp = nbr[(size_t)9 * B + 1 + 2 * MU];
    cx<float> hv[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) hv[c] = mk(0.f, 0.f);
    const float4* wl = nullptr;
    if (l == kSapB - 1) {
      int y0 = x0, y1 = x1, y2 = x2, y3 = x3;
      bool neg;
      geo_step<MU, +1>(g, y0, y1, y2, y3, neg);
      const int bs = sap_bsite<false>(sb, y0, y1, y2, y3);
      hop_term<MU, false>(hv, w, u, neg);
#pragma unroll
      for (int c = 0; c < 12; ++c) hv[c] = -0.5f * hv[c];
      wl = W + (size_t)(bs / kSapSites) * bsz + (bs % kSapSites);
    }
    dfl_project<false>(red, wl, hv, ns, A + (((size_t)Bp * 9 + 2 + 2 * MU) * ns + k) * ns, 1);
  }
  {  // -MU: y = x - MU in B' = B - MU gets -(1/2) (1 - g_MU) U(y, MU) w(x)
    const int Bp = nbr[(size_t)9 * B + 2 + 2 * MU];
    cx<float> hv[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) hv[c] = mk(0.f, 0.f);
    const float4* wl = nullptr;
    if (l == 0) {
      int y0 = x0, y1 = x1, y2 = x2, y3 = x3;
      bool neg;
      geo_step<MU, -1>(g, y0, y1, y2, y3, neg);
      const int bs = sap_bsite<false>(sb, y0, y1, y2, y3);
      cx<float> uy[9];
      const float2* vb = sap_blk<36>(Vb, bs / kSapSites) + MU * 9 * kSapSites + (bs % kSapSites);
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        float2 a = vb[c * kSapSites];
        uy[c] = mk(a.x, a.y);
      }
      hop_term<MU, true>(hv, w, uy, neg);
#pragma unroll
      for (int c = 0; c < 12; ++c) hv[c] = -0.5f * hv[c];
      wl = W + (size_t)(bs / kSapSites) * bsz + (bs % kSapSites);
    }
    dfl_project<false>(red, wl, hv, ns, A + (((size_t)Bp * 9 + 1 + 2 * MU) * ns + k) * ns, 1);
  }
}

// The little operator, one workgroup per block B and its basis vectors w_k:
// the in-block part of D w_k (LDS exchange) projected on B's basis, the face
// hops on the neighbours' bases.
__global__ __launch_bounds__(kSapSites) void k_dfl_little(Geo g, SapGeo sb, int ns, const float4* __restrict__ W,
                                                          const float2* __restrict__ Vb,
                                                          const float4* __restrict__ Cb, const int* __restrict__ nbr,
                                                          float2* __restrict__ A) {
  __shared__ SapLds L;
  __shared__ float2 red[kSapSites / 64][kDflMaxNs];
  const int B = blockIdx.x, t = threadIdx.x;
  int x0, x1, x2, x3, p;
  size_t h;
  dfl_site(g, sb, B, t, x0, x1, x2, x3, p, h);
  const int l0 = t >> 6, l1 = (t >> 4) & 3, l2 = (t >> 2) & 3, l3 = t & 3;
  cx<float> U[4][9];
  {
    const float2* vb = sap_blk<36>(Vb, B) + t;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        float2 v = vb[(mu * 9 + c) * kSapSites];
        U[mu][c] = mk(v.x, v.y);
      }
  }
  const float4* cb = sap_blk<18>(Cb, B) + t;
  const size_t bsz = (size_t)ns * 6 * kSapSites;
  const float4* wb = W + (size_t)B * bsz;
  for (int k = 0; k < ns; ++k) {
    cx<float> w[12], acc[12], v[12];
    sp_load(wb + (size_t)k * 6 * kSapSites, kSapSites, t, w);
    sap_publish<false>(L, w, U);
    __syncthreads();
    sap_gather<false>(L, U, acc);
    sap_clover<kSapSites>(cb, w, v);
#pragma unroll
    for (int c = 0; c < 12; ++c) v[c] = v[c] - 0.5f * acc[c];
    // (the projections' barriers also separate these reads from the next publish)
    dfl_project<false>(red, wb + t, v, ns, A + ((size_t)B * 9 * ns + k) * ns, 1);
    dfl_faces<0>(g, sb, red, B, x0, x1, x2, x3, l0, w, U[0], W, Vb, nbr, ns, k, A);
    dfl_faces<1>(g, sb, red, B, x0, x1, x2, x3, l1, w, U[1], W, Vb, nbr, ns, k, A);
    dfl_faces<2>(g, sb, red, B, x0, x1, x2, x3, l2, w, U[2], W, Vb, nbr, ns, k, A);
    dfl_faces<3>(g, sb, red, B, x0, x1, x2, x3, l3, w, U[3], W, Vb, nbr, ns, k, A);
  }
}

// W^+ of the field (f_e, f_o) (f_o null: zero) into c [B][ns].
__global__ __launch_bounds__(kSapSites) void k_dfl_restrict(Geo g, SapGeo sb, int ns, const float4* __restrict__ W,
                                                            const float4* __restrict__ f_e,
                                                            const float4* __restrict__ f_o, float2* __restrict__ c) {
  __shared__ float2 red[kSapSites / 64][kDflMaxNs];
  const int B = blockIdx.x, t = threadIdx.x;
  int x0, x1, x2, x3, p;
  size_t h;
  dfl_site(g, sb, B, t, x0, x1, x2, x3, p, h);
  cx<float> f[12];
  if (p == 0 || f_o) {
    sp_load(p ? f_o : f_e, g.Ve, h, f);
  } else {
#pragma unroll
    for (int k = 0; k < 12; ++k) f[k] = mk(0.f, 0.f);
  }
  dfl_project<true>(red, W + (size_t)B * ns * 6 * kSapSites + t, f, ns, c + (size_t)B * ns, 1);
}

// out = W c, both halves of an FP32 full field.
__global__ __launch_bounds__(kSapSites) void k_dfl_prolong(Geo g, SapGeo sb, int ns, const float4* __restrict__ W,
                                                           const float2* __restrict__ c, float4* __restrict__ out_e,
                                                           float4* __restrict__ out_o) {
  const int B = blockIdx.x, t = threadIdx.x;
  int x0, x1, x2, x3, p;
  size_t h;
  dfl_site(g, sb, B, t, x0, x1, x2, x3, p, h);
  const float4* wb = W + (size_t)B * ns * 6 * kSapSites + t;
  cx<float> o[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) o[k] = mk(0.f, 0.f);
#pragma unroll 4
  for (int k = 0; k < ns; ++k) {
    const float2 ck = c[(size_t)B * ns + k];
    const cx<float> a = mk(ck.x, ck.y);
    cx<float> w[12];
    dfl_wload(wb + (size_t)k * 6 * kSapSites, w);
#pragma unroll
    for (int m = 0; m < 12; ++m) o[m] = o[m] + a * w[m];
  }
  sp_store(p ? out_o : out_e, g.Ve, h, o);
}

// y = A x (one thread per coarse row); z = x when given
__global__ __launch_bounds__(QXD_BLOCK) void k_dfl_cmv(int nblk, int ns, const float2* __restrict__ A,
                                                       const int* __restrict__ nbr, const float2* __restrict__ x,
                                                       float2* __restrict__ y, float2* __restrict__ z) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (size_t)nblk * ns) return;
  const int B = (int)(i / ns), l = (int)(i % ns);
  float re = 0.f, im = 0.f;
  for (int n = 0; n < 9; ++n) {
    const float2* a = A + ((size_t)B * 9 + n) * ns * ns + l;
    const float2* xv = x + (size_t)nbr[(size_t)9 * B + n] * ns;
    for (int k = 0; k < ns; ++k) {
      const float2 av = a[(size_t)k * ns], xk = xv[k];
      re += av.x * xk.x - av.y * xk.y;
      im += av.x * xk.y + av.y * xk.x;
    }
  }
  y[i] = make_float2(re, im);
  if (z) z[i] = x[i];
}

// t_e = r_e - t_e, t_o = -t_o (t holds D psi on entry)
__global__ __launch_bounds__(QXD_BLOCK) void k_dfl_sub(size_t n, const float4* __restrict__ r_e,
                                                       float4* __restrict__ t) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < 2 * n; i += (size_t)gridDim.x * blockDim.x) {
    const float4 d = t[i];
    if (i < n) {
      const float4 a = r_e[i];
      t[i] = make_float4(a.x - d.x, a.y - d.y, a.z - d.z, a.w - d.w);
    } else {
      t[i] = make_float4(-d.x, -d.y, -d.z, -d.w);
    }
  }
}

// out = a + b
__global__ __launch_bounds__(QXD_BLOCK) void k_dfl_add(size_t n, const float4* __restrict__ a,
                                                       const float4* __restrict__ b, float4* __restrict__ out) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float4 u = a[i], v = b[i];
    out[i] = make_float4(u.x + v.x, u.y + v.y, u.z + v.z, u.w + v.w);
  }
}

// v = u / sqrt(scal[slot])
__global__ __launch_bounds__(QXD_BLOCK) void k_dfl_scale(size_t n, const float4* __restrict__ u,
                                                         float4* __restrict__ v, const double* __restrict__ scal,
                                                         int slot) {
  const float sc = (float)(1.0 / sqrt(scal[slot]));
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const float4 a = u[i];
    v[i] = make_float4(sc * a.x, sc * a.y, sc * a.z, sc * a.w);
  }
}

// c = e_k on every block
__global__ __launch_bounds__(QXD_BLOCK) void k_zero_coarse_unit(int nblk, int ns, int k, float2* __restrict__ c) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < (size_t)nblk * ns) c[i] = make_float2((int)(i % ns) == k ? 1.f : 0.f, 0.f);
}

int dfl_grid(size_t n) { return (int)std::min<size_t>(QXD_NRED, (n + QXD_BLOCK - 1) / QXD_BLOCK); }

// nc GCR steps on A c = b from c = 0, no restart; every scalar stays on the
// device.  The coarse vectors are viewed as float4 pairs of complex numbers.
qxd_status dfl_coarse(qxd_handle* h, qxd_dfl* d, int nc, hipStream_t s) {
  const size_t N = (size_t)d->nblk * d->ns, n4 = N / 2;
  auto v4 = [](float2* p) { return reinterpret_cast<float4*>(p); };
  blas_zero<float4>(v4(d->cx), n4, s);
  QXD_HIP(hipMemcpyAsync(d->cr, d->cb, N * sizeof(float2), hipMemcpyDeviceToDevice, s));
  const int g = (int)((N + QXD_BLOCK - 1) / QXD_BLOCK);
  for (int k = 0; k < nc; ++k) {
    float2* z = d->cz + k * N;
    float2* w = d->cw + k * N;
    hipLaunchKernelGGL(k_dfl_cmv, dim3(g), dim3(QXD_BLOCK), 0, s, d->nblk, d->ns, d->A, d->nbr, d->cr, w, z);
    if (k == 0) {
      blas_norm2<float4>(h, v4(w), n4, h->scal + S_DN, s);
    } else {
      Ptrs pw{}, pz{};
      for (int j = 0; j < k; ++j) {
        pw.p[j] = d->cw + j * N;
        pz.p[j] = d->cz + j * N;
      }
      blas_mdot<float4>(h, pw, k, v4(w), n4, h->scal + S_DC, s);
      blas_mupdate<float4>(h, v4(w), pw, k, h->scal + S_DC, n4, h->scal + S_DN, s);
      blas_mupdate<float4>(h, v4(z), pz, k, h->scal + S_DC, n4, h->scal + S_DY, s);
    }
    blas_scale_cdot<float4>(h, v4(w), v4(d->cr), n4, S_DN, h->scal + S_DA, s);
    blas_scale_cdot<float4>(h, v4(z), v4(d->cr), n4, S_DN, h->scal + S_DX, s);
    blas_r_update<float4>(h, v4(d->cr), v4(w), n4, S_DA, h->scal + S_DY, s);
    Ptrs pz1{};
    pz1.p[0] = z;
    blas_multi_axpy<float4>(h, v4(d->cx), pz1, 1, h->scal + S_DA, n4, s);
  }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

// The handle's lattice must be the one the object was made for.
bool dfl_same_lattice(const qxd_handle* h, const qxd_dfl* d) {
  const Geo &a = h->geo, &b = d->geo;
  return a.Le0 == b.Le0 && a.Le1 == b.Le1 && a.Le2 == b.Le2 && a.Le3 == b.Le3 && a.L1 == b.L1 && a.cstar == b.cstar &&
         a.tanti == b.tanti;
}

qxd_status dfl_build_little(qxd_handle* h, qxd_dfl* d, hipStream_t s) {
  const float2* Vb;
  const float4* Cb;
  SapGeo sb;
  QXD_TRY(sap_blocks(h, 0, &Vb, &Cb, &sb, s));
  hipLaunchKernelGGL(k_dfl_little, dim3(d->nblk), dim3(kSapSites), 0, s, h->geo, d->sb, d->ns, d->W, Vb, Cb, d->nbr,
                     d->A);
  QXD_HIP(hipGetLastError());
  d->op = h;
  d->gen = h->setup_gen;
  return QXD_OK;
}

}  // namespace

qxd_status dfl_apply_internal(qxd_handle* h, qxd_dfl* d, int nc, int ncy, int nmr, int eo, float4* out_e,
                              const float4* in_e, hipStream_t s) {
  if (nc < 1 || nc > kDflMaxNc || !dfl_same_lattice(h, d)) return QXD_EINVAL;
  if (!d->has_basis || d->op != h || d->gen != h->setup_gen) return QXD_ESTATE;
  const Geo& g = h->geo;
  const size_t half = (size_t)6 * h->Ve;
  hipLaunchKernelGGL(k_dfl_restrict, dim3(d->nblk), dim3(kSapSites), 0, s, g, d->sb, d->ns, d->W, in_e,
                     (const float4*)nullptr, d->cb);
  QXD_TRY(dfl_coarse(h, d, nc, s));
  hipLaunchKernelGGL(k_dfl_prolong, dim3(d->nblk), dim3(kSapSites), 0, s, g, d->sb, d->ns, d->W, d->cx, d->psi,
                     d->psi + half);
  QXD_TRY(qxd_dw_apply(h, QXD_F32, d->t, d->psi, s));
  hipLaunchKernelGGL(k_dfl_sub, dim3(dfl_grid(2 * half)), dim3(QXD_BLOCK), 0, s, half, in_e, d->t);
  QXD_TRY(sap_apply_internal(h, ncy, nmr, eo, d->xs, d->t, s, d->t + half, nullptr));
  hipLaunchKernelGGL(k_dfl_add, dim3(dfl_grid(half)), dim3(QXD_BLOCK), 0, s, half, d->psi, d->xs, out_e);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_create(qxd_handle* h, int ns, qxd_dfl** out) {
  if (!h || !out || ns < 1 || ns > kDflMaxNs) return QXD_EINVAL;
  *out = nullptr;
  if (!sap_supported(h)) return QXD_EGEOM;
  qxd_dfl* d = new (std::nothrow) qxd_dfl;
  if (!d) return QXD_ENOMEM;
  const Geo& g = h->geo;
  d->ns = ns;
  d->geo = g;
  d->nblk = (g.Le0 / kSapB) * (g.Le1 / kSapB) * (g.Le2 / kSapB) * (g.Le3 / kSapB);
  d->sb = SapGeo{g.Le1 / kSapB, g.Le2 / kSapB, g.Le3 / kSapB, d->nblk / 2};
  const size_t V = (size_t)h->V, N = (size_t)d->nblk * ns;
  bool ok = dev_alloc(&d->W, V * ns * 6 * sizeof(float4)) &&
            dev_alloc(&d->A, N * 9 * ns * sizeof(float2)) &&
            dev_alloc(&d->nbr, (size_t)d->nblk * 9 * sizeof(int)) &&
            dev_alloc(&d->cb, N * sizeof(float2)) && dev_alloc(&d->cx, N * sizeof(float2)) &&
            dev_alloc(&d->cr, N * sizeof(float2)) &&
            dev_alloc(&d->cz, kDflMaxNc * N * sizeof(float2)) &&
            dev_alloc(&d->cw, kDflMaxNc * N * sizeof(float2)) &&
            dev_alloc(&d->psi, V * 6 * sizeof(float4)) &&
            dev_alloc(&d->t, V * 6 * sizeof(float4)) &&
            dev_alloc(&d->xs, V * 3 * sizeof(float4));
  if (!ok) {
    qxd_dfl_destroy(d);
    return QXD_ENOMEM;
  }
  hipLaunchKernelGGL(k_dfl_nbr, dim3((d->nblk + 127) / 128), dim3(128), 0, 0, g, d->sb, d->nblk, d->nbr);
  if (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
    qxd_dfl_destroy(d);
    return QXD_EHIP;
  }
  *out = d;
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_destroy(qxd_dfl* d) {
  if (!d) return QXD_EINVAL;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {d->W, d->A, d->nbr, d->cb, d->cx, d->cr, d->cz, d->cw, d->psi, d->t, d->xs};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete d;
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_generate(qxd_handle* h, qxd_dfl* d, void* v, int nit, int ncy, int nmr, void* stream) {
  if (!h || !d || !v || nit < 0 || nit > 100 || !dfl_same_lattice(h, d)) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  const size_t full = (size_t)12 * h->Ve, half = full / 2;
  float4* vs = static_cast<float4*>(v);
  for (int k = 0; k < d->ns; ++k) {
    float4* vk = vs + k * full;
    for (int it = 0; it < nit; ++it) {
      QXD_TRY(sap_apply_internal(h, ncy, nmr, 0, d->psi, vk, s, vk + half, d->psi + half));
      blas_norm2<float4>(h, d->psi, full, h->scal + S_DY, s);
      hipLaunchKernelGGL(k_dfl_scale, dim3(dfl_grid(full)), dim3(QXD_BLOCK), 0, s, full, d->psi, vk, h->scal, S_DY);
    }
  }
  hipLaunchKernelGGL(k_dfl_orth, dim3(d->nblk), dim3(kSapSites), 0, s, h->geo, d->sb, d->ns, vs, full, d->W);
  QXD_HIP(hipGetLastError());
  d->has_basis = true;
  QXD_TRY(dfl_build_little(h, d, s));
  QXD_HIP(hipStreamSynchronize(s));
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_little(qxd_handle* h, qxd_dfl* d, void* stream) {
  if (!h || !d || !dfl_same_lattice(h, d)) return QXD_EINVAL;
  if (!d->has_basis || !h->has_inverse) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  QXD_TRY(dfl_build_little(h, d, s));
  QXD_HIP(hipStreamSynchronize(s));
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_apply(qxd_handle* h, qxd_dfl* d, int nc, int ncy, int nmr, int eo, void* out_e,
                                    const void* in_e, void* stream) {
  if (!h || !d || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  if (ncy < 1 || nmr < 1 || ncy > 64 || nmr > 64 || (eo != 0 && eo != 1)) return QXD_EINVAL;
  return dfl_apply_internal(h, d, nc, ncy, nmr, eo, (float4*)out_e, (const float4*)in_e, as_stream(stream));
}

extern "C" qxd_status qxd_dfl_basis(qxd_handle* h, qxd_dfl* d, int k, void* out, void* stream) {
  if (!h || !d || !out || k < 0 || k >= d->ns || !dfl_same_lattice(h, d)) return QXD_EINVAL;
  if (!d->has_basis) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  // the basis vector w_{B,k} of every block: W c with c = e_k on every block
  hipLaunchKernelGGL(k_zero_coarse_unit, dim3(dfl_grid((size_t)d->nblk * d->ns)), dim3(QXD_BLOCK), 0, s, d->nblk,
                     d->ns, k, d->cx);
  const size_t half = (size_t)6 * h->Ve;
  hipLaunchKernelGGL(k_dfl_prolong, dim3(d->nblk), dim3(kSapSites), 0, s, h->geo, d->sb, d->ns, d->W, d->cx,
                     (float4*)out, (float4*)out + half);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_little_get(qxd_dfl* d, float* A, int* nbr) {
  if (!d || !A || !nbr) return QXD_EINVAL;
  if (!d->has_basis) return QXD_ESTATE;
  const size_t N = (size_t)d->nblk * d->ns;
  QXD_HIP(hipMemcpy(A, d->A, N * 9 * d->ns * sizeof(float2), hipMemcpyDeviceToHost));
  QXD_HIP(hipMemcpy(nbr, d->nbr, (size_t)d->nblk * 9 * sizeof(int), hipMemcpyDeviceToHost));
  return QXD_OK;
}

extern "C" qxd_status qxd_dfl_size(const qxd_dfl* d, int* nblk, int* ns) {
  if (!d) return QXD_EINVAL;
  if (nblk) *nblk = d->nblk;
  if (ns) *ns = d->ns;
  return QXD_OK;
}
