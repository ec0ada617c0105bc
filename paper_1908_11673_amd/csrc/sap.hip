// Schwarz alternating procedure (SAP): the paper's domain-decomposition
// preconditioner for GCR (Sec. 4.4, SAP+GCR), on the full Wilson-clover
// operator in FP32.
//
// The extended lattice is cut into 4^4 blocks coloured by the parity of their
// block coordinates.  A half cycle on colour c: on every block B of colour c,
// r_B = (eta - D x)_B, then nmr minimal-residual steps on the block operator D_B
// (D restricted to B, hops leaving B dropped) from e = 0, and x_B += e.  Blocks
// of one colour are never neighbours, so a half cycle is one launch with one
// workgroup per block and no races: x is read outside the block (other colour)
// and written inside it.  ncy cycles (colour 0 then 1) from x = 0 give M eta.
//
// A workgroup of 256 threads owns one block, one thread per site; a site keeps
// its four forward links in registers.  Each minimal-residual step every site
// publishes rho (24.6 kB of LDS) and, for each direction, the backward hop it
// owes its forward neighbour, (1 + g_mu) U^+ rho as two colour vectors (49.2 kB):
// 74 kB of LDS per block, so two blocks share a CU.  The block reductions of the
// step go through LDS.  The residual at entry
// (the only part that reads outside the block) is a site-parallel kernel of its
// own, run before each half cycle but the first.
#include "blas.hpp"
#include "wilson_site.hpp"

namespace {

constexpr int kSapB = 4;                            // block extent
constexpr int kSapSites = kSapB * kSapB * kSapB * kSapB;  // 256: one thread per site

struct SapGeo {
  int nb1, nb2, nb3;  // blocks along x1, x2, x3 (nb3 even)
};

// Plain (cached) loads: every step of a block solve reads the clover blocks again.
__device__ __forceinline__ void sap_clover(const float4* __restrict__ C, size_t Ve, int h, const cx<float> in[12],
                                           cx<float> out[12]) {
  float r[72];
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    float4 v = C[k * Ve + h];
    r[4 * k] = v.x;
    r[4 * k + 1] = v.y;
    r[4 * k + 2] = v.z;
    r[4 * k + 3] = v.w;
  }
  herm6_mul<float>(r, in, out);
  herm6_mul<float>(r + 36, in + 6, out + 6);
}

// The backward hop that site t contributes to its forward neighbour along MU:
// (1 + g_MU) U(t, MU)^+ rho(t), kept as the two multiplied colour vectors.
template <int MU>
__device__ __forceinline__ void sap_send(float2 (*bw_s)[6][kSapSites], int t, const cx<float> rho[12],
                                         const cx<float> u[9]) {
  cx<float> h0[3], h1[3], w0[3], w1[3];
  spin_project<MU, false>(rho, h0, h1);
  colour_mul<false>(u, h0, h1, w0, w1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bw_s[MU][a][t] = make_float2(w0[a].re, w0[a].im);
    bw_s[MU][3 + a][t] = make_float2(w1[a].re, w1[a].im);
  }
}

// Both in-block hops along MU at site t (local coordinate l along MU, strides
// 64, 16, 4, 1): forward with the site's own link and the neighbour's rho,
// backward as sent by the neighbour.
template <int MU>
__device__ __forceinline__ void sap_recv(const float4 (*rho_s)[kSapSites], const float2 (*bw_s)[6][kSapSites], int t,
                                         int l, const cx<float> u[9], cx<float> acc[12]) {
  constexpr int st = MU == 0 ? 64 : MU == 1 ? 16 : MU == 2 ? 4 : 1;
  if (l < kSapB - 1) {
    cx<float> s[12];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float4 v = rho_s[j][t + st];
      s[2 * j] = mk(v.x, v.y);
      s[2 * j + 1] = mk(v.z, v.w);
    }
    hop_term<MU, true>(acc, s, u, false);
  }
  if (l > 0) {
    cx<float> w0[3], w1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float2 v0 = bw_s[MU][a][t - st], v1 = bw_s[MU][3 + a][t - st];
      w0[a] = mk(v0.x, v0.y);
      w1[a] = mk(v1.x, v1.y);
    }
    spin_rebuild_add<MU, false>(acc, w0, w1);
  }
}

__device__ __forceinline__ float sap_wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Residual of the blocks of `colour`: r = eta - D x at their sites (one
// workgroup per block, one thread per site, the same site order as the block
// solver), into the FP32 half fields r_e, r_o.  A site-parallel kernel of its
// own, so that the neighbour loads of D run at full occupancy.
__global__ __launch_bounds__(kSapSites) void k_sap_resid(Geo g, SapGeo sb, int colour,
                                                         const float4* __restrict__ eta_e,
                                                         const float4* __restrict__ x_e,
                                                         const float4* __restrict__ x_o,
                                                         const float2* __restrict__ V32,
                                                         const float4* __restrict__ He,
                                                         const float4* __restrict__ Ho, float4* __restrict__ r_e,
                                                         float4* __restrict__ r_o) {
  const int half3 = sb.nb3 >> 1;
  int k3 = blockIdx.x % half3, line = blockIdx.x / half3;
  const int c2 = line % sb.nb2;
  line /= sb.nb2;
  const int c1 = line % sb.nb1, c0 = line / sb.nb1;
  const int c3 = 2 * k3 + ((c0 + c1 + c2 + colour) & 1);
  const int t = threadIdx.x;
  const int x0 = kSapB * c0 + (t >> 6), x1 = kSapB * c1 + ((t >> 4) & 3), x2 = kSapB * c2 + ((t >> 2) & 3),
            x3 = kSapB * c3 + (t & 3);
  const int p = (x0 + x1 + x2 + x3) & 1;
  const int h = geo_half(g, x0, x1, x2, x3);
  const size_t Ve = g.Ve;
  const float2* Vp = V32 + (size_t)p * 36 * Ve;
  const float2* Vq = V32 + (size_t)(1 - p) * 36 * Ve;
  cx<float> r[12], xs[12], hx[12], dx[12];
  if (p == 0) {
    sp_load(eta_e, Ve, h, r);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) r[c] = mk(0.f, 0.f);
  }
  sp_load(p ? x_o : x_e, Ve, h, xs);
  hop_site<false, float>(g, p, h, p ? x_e : x_o, Vp, Vq, hx);
  clover_mul<float>(p ? Ho : He, Ve, h, xs, dx);
#pragma unroll
  for (int c = 0; c < 12; ++c) r[c] = r[c] - (dx[c] - 0.5f * hx[c]);
  sp_store(p ? r_o : r_e, Ve, h, r);
}

// One half cycle on the blocks of `colour`: block solves of the residual
// (r_e, r_o) added to x = (x_e, x_o), FP32 half fields.  XZERO: x is zero on
// entry (first half cycle) and the residual is the source, r_e = eta (its odd
// half is zero and r_o is not read).
template <bool XZERO>
__global__ __launch_bounds__(kSapSites, 2) void k_sap_half(Geo g, SapGeo sb, int colour, int nmr,
                                                           const float4* __restrict__ r_e,
                                                           const float4* __restrict__ r_o,
                                                           float4* __restrict__ x_e, float4* __restrict__ x_o,
                                                           const float2* __restrict__ V32,
                                                           const float4* __restrict__ He,
                                                           const float4* __restrict__ Ho) {
  __shared__ float4 rho_s[6][kSapSites];
  __shared__ float2 bw_s[4][6][kSapSites];
  __shared__ float red_s[3][kSapSites / 64];
  // the blockIdx-th block of this colour: along x3 the colours alternate
  const int half3 = sb.nb3 >> 1;
  int k3 = blockIdx.x % half3, line = blockIdx.x / half3;
  const int c2 = line % sb.nb2;
  line /= sb.nb2;
  const int c1 = line % sb.nb1, c0 = line / sb.nb1;
  const int c3 = 2 * k3 + ((c0 + c1 + c2 + colour) & 1);
  const int t = threadIdx.x;
  const int l0 = t >> 6, l1 = (t >> 4) & 3, l2 = (t >> 2) & 3, l3 = t & 3;
  const int x0 = kSapB * c0 + l0, x1 = kSapB * c1 + l1, x2 = kSapB * c2 + l2, x3 = kSapB * c3 + l3;
  const int p = (x0 + x1 + x2 + x3) & 1;
  const int h = geo_half(g, x0, x1, x2, x3);
  const size_t Ve = g.Ve;
  const float2* Vp = V32 + (size_t)p * 36 * Ve;
  const float4* Hp = p ? Ho : He;
  float4* xp = p ? x_o : x_e;

  // the site's four forward links stay in registers for the whole solve
  cx<float> U[4][9];
#pragma unroll
  for (int mu = 0; mu < 4; ++mu)
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 v = Vp[(mu * 9 + k) * Ve + h];
      U[mu][k] = mk(v.x, v.y);
    }
  // the block's residual: eta itself while x = 0 (r_e = eta, r_o unused),
  // else from k_sap_resid
  cx<float> rho[12];
  if (p == 0 || !XZERO) {
    sp_load(p ? r_o : r_e, Ve, h, rho);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = mk(0.f, 0.f);
  }
  cx<float> e[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) e[c] = mk(0.f, 0.f);
  const int wave = t >> 6, lane = t & 63;
  for (int step = 0; step < nmr; ++step) {
    // publish rho and the backward hops this site owes its forward neighbours
    // (every read of the previous step's values came before its reduction barrier)
#pragma unroll
    for (int j = 0; j < 6; ++j)
      rho_s[j][t] = make_float4(rho[2 * j].re, rho[2 * j].im, rho[2 * j + 1].re, rho[2 * j + 1].im);
    if (l0 < kSapB - 1) sap_send<0>(bw_s, t, rho, U[0]);
    if (l1 < kSapB - 1) sap_send<1>(bw_s, t, rho, U[1]);
    if (l2 < kSapB - 1) sap_send<2>(bw_s, t, rho, U[2]);
    if (l3 < kSapB - 1) sap_send<3>(bw_s, t, rho, U[3]);
    __syncthreads();
    // v = D_B rho = H rho - (1/2) (in-block hops)
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = mk(0.f, 0.f);
    sap_recv<0>(rho_s, bw_s, t, l0, U[0], acc);
    sap_recv<1>(rho_s, bw_s, t, l1, U[1], acc);
    sap_recv<2>(rho_s, bw_s, t, l2, U[2], acc);
    sap_recv<3>(rho_s, bw_s, t, l3, U[3], acc);
    cx<float> v[12];
    sap_clover(Hp, Ve, h, rho, v);
    float are = 0.f, aim = 0.f, nn = 0.f;
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      v[c] = v[c] - 0.5f * acc[c];
      cx<float> vr = cmul_conj(v[c], rho[c]);  // conj(v) rho
      are += vr.re;
      aim += vr.im;
      nn += norm2(v[c]);
    }
    are = sap_wave_sum(are);
    aim = sap_wave_sum(aim);
    nn = sap_wave_sum(nn);
    if (lane == 0) {
      red_s[0][wave] = are;
      red_s[1][wave] = aim;
      red_s[2][wave] = nn;
    }
    __syncthreads();
    are = aim = nn = 0.f;
#pragma unroll
    for (int w = 0; w < kSapSites / 64; ++w) {
      are += red_s[0][w];
      aim += red_s[1][w];
      nn += red_s[2][w];
    }
    // alpha = (v, rho) / (v, v); a block whose residual vanished stays put
    const cx<float> alpha = nn > 0.f ? mk(are / nn, aim / nn) : mk(0.f, 0.f);
#pragma unroll
    for (int c = 0; c < 12; ++c) {
      e[c] = e[c] + alpha * rho[c];
      rho[c] = rho[c] - alpha * v[c];
    }
  }
  if (!XZERO) {
    cx<float> xs[12];
    sp_load(xp, Ve, h, xs);
#pragma unroll
    for (int c = 0; c < 12; ++c) e[c] = e[c] + xs[c];
  }
  sp_store(xp, Ve, h, e);
}

enum { W_SAP_XO = 13, W_SAP_RE, W_SAP_RO };  // workspace roles (free in the solvers' table)

}  // namespace

// Geometry the block colouring supports: an even number (at least two) of 4^4
// blocks along every direction and, with C* in k >= 2, an x1 shift of L1 that
// moves an even number of blocks (so neighbours across a shifted boundary still
// differ in colour).
bool sap_supported(const qxd_handle* h) {
  const Geo& g = h->geo;
  if (g.Le0 % (2 * kSapB) || g.Le1 % (2 * kSapB) || g.Le2 % (2 * kSapB) || g.Le3 % (2 * kSapB)) return false;
  return g.cstar < 2 || (g.L1 / kSapB) % 2 == 0;
}

qxd_status sap_apply_internal(qxd_handle* h, int ncy, int nmr, float4* out_e, const float4* in_e, hipStream_t s) {
  if (ncy < 1 || nmr < 1 || ncy > 64 || nmr > 64) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  if (!sap_supported(h)) return QXD_EGEOM;
  const size_t n32 = (size_t)6 * h->Ve;
  float4* xo = (float4*)ws_get(h, W_SAP_XO, n32 * sizeof(float4));
  float4* re = (float4*)ws_get(h, W_SAP_RE, n32 * sizeof(float4));
  float4* ro = (float4*)ws_get(h, W_SAP_RO, n32 * sizeof(float4));
  if (!xo || !re || !ro) return QXD_ENOMEM;
  // x = 0 on both halves: the first half cycle writes the colour-0 blocks only
  blas_zero<float4>(out_e, n32, s);
  blas_zero<float4>(xo, n32, s);
  SapGeo sb{h->geo.Le1 / kSapB, h->geo.Le2 / kSapB, h->geo.Le3 / kSapB};
  const int nblk = (h->geo.Le0 / kSapB) * sb.nb1 * sb.nb2 * sb.nb3;
  dim3 grid(nblk / 2), blk(kSapSites);
  const float2* V32 = reinterpret_cast<const float2*>(h->V32);
  const float4* He = reinterpret_cast<const float4*>(h->He32);
  const float4* Ho = reinterpret_cast<const float4*>(h->Ho32);
  for (int cy = 0; cy < ncy; ++cy)
    for (int colour = 0; colour < 2; ++colour) {
      if (cy == 0 && colour == 0) {
        hipLaunchKernelGGL(k_sap_half<true>, grid, blk, 0, s, h->geo, sb, colour, nmr, in_e, nullptr, out_e, xo, V32,
                           He, Ho);
      } else {
        hipLaunchKernelGGL(k_sap_resid, grid, blk, 0, s, h->geo, sb, colour, in_e, out_e, xo, V32, He, Ho, re, ro);
        hipLaunchKernelGGL(k_sap_half<false>, grid, blk, 0, s, h->geo, sb, colour, nmr, re, ro, out_e, xo, V32, He,
                           Ho);
      }
    }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_sap_apply(qxd_handle* h, int ncy, int nmr, void* out_e, const void* in_e, void* stream) {
  if (!h || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  return sap_apply_internal(h, ncy, nmr, (float4*)out_e, (const float4*)in_e, as_stream(stream));
}
