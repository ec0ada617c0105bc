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
// A workgroup holds its block in LDS: the 256 sites' forward links (73.7 kB) and
// the current rho (24.6 kB); each thread owns one site, keeps its clover blocks
// in registers, and forms D_B rho from its in-block neighbours; the block
// reductions of the minimal-residual step go through LDS.  Only the residual
// at entry touches sites outside the block.
#include "blas.hpp"
#include "wilson_site.hpp"

namespace {

constexpr int kSapB = 4;                            // block extent
constexpr int kSapSites = kSapB * kSapB * kSapB * kSapB;  // 256: one thread per site

struct SapGeo {
  int nb1, nb2, nb3;  // blocks along x1, x2, x3 (nb3 even)
};

// Add the in-block hops along MU at local site t (strides 64, 16, 4, 1).
template <int MU>
__device__ __forceinline__ void sap_hop(const float4 (*rho_s)[kSapSites], const float2 (*lk_s)[9][kSapSites], int t,
                                        int l, cx<float> acc[12]) {
  constexpr int st = MU == 0 ? 64 : MU == 1 ? 16 : MU == 2 ? 4 : 1;
  cx<float> s[12], u[9];
  if (l < kSapB - 1) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float4 v = rho_s[j][t + st];
      s[2 * j] = mk(v.x, v.y);
      s[2 * j + 1] = mk(v.z, v.w);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 v = lk_s[MU][k][t];
      u[k] = mk(v.x, v.y);
    }
    hop_term<MU, true>(acc, s, u, false);
  }
  if (l > 0) {
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float4 v = rho_s[j][t - st];
      s[2 * j] = mk(v.x, v.y);
      s[2 * j + 1] = mk(v.z, v.w);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 v = lk_s[MU][k][t - st];
      u[k] = mk(v.x, v.y);
    }
    hop_term<MU, false>(acc, s, u, false);
  }
}

__device__ __forceinline__ float sap_wave_sum(float v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// One half cycle on the blocks of `colour`.  eta: even half of the source (its
// odd half is zero); x = (x_e, x_o), FP32 half fields.  XZERO: x is zero on
// entry (first half cycle), so the residual is eta itself.
template <bool XZERO>
__global__ __launch_bounds__(kSapSites) void k_sap_half(Geo g, SapGeo sb, int colour, int nmr,
                                                        const float4* __restrict__ eta_e, float4* __restrict__ x_e,
                                                        float4* __restrict__ x_o, const float2* __restrict__ V32,
                                                        const float4* __restrict__ He, const float4* __restrict__ Ho) {
  __shared__ float4 rho_s[6][kSapSites];
  __shared__ float2 lk_s[4][9][kSapSites];
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
  const float2* Vq = V32 + (size_t)(1 - p) * 36 * Ve;
  float4* xp = p ? x_o : x_e;
  const float4* xq = p ? x_e : x_o;

  float cl[72];
  cl_load(p ? Ho : He, Ve, h, cl);
  cx<float> rho[12];
  if (p == 0) {
    sp_load(eta_e, Ve, h, rho);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = mk(0.f, 0.f);
  }
  cx<float> xs[12];
  if (!XZERO) {
    // r = eta - D x at this site (neighbours anywhere on the lattice)
    sp_load(xp, Ve, h, xs);
    cx<float> hx[12], dx[12];
    hop_site<false, float>(g, p, h, xq, Vp, Vq, hx);
    herm6_mul<float>(cl, xs, dx);
    herm6_mul<float>(cl + 36, xs + 6, dx + 6);
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = rho[c] - (dx[c] - 0.5f * hx[c]);
  }
  {
    cx<float> u[9];
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
      lk_load(Vp, Ve, mu, h, u);
#pragma unroll
      for (int k = 0; k < 9; ++k) lk_s[mu][k][t] = make_float2(u[k].re, u[k].im);
    }
  }
  cx<float> e[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) e[c] = mk(0.f, 0.f);
  const int wave = t >> 6, lane = t & 63;
  for (int step = 0; step < nmr; ++step) {
    __syncthreads();  // the previous step's reads of rho_s are done
#pragma unroll
    for (int j = 0; j < 6; ++j)
      rho_s[j][t] = make_float4(rho[2 * j].re, rho[2 * j].im, rho[2 * j + 1].re, rho[2 * j + 1].im);
    __syncthreads();
    // v = D_B rho = H rho - (1/2) (in-block hops)
    cx<float> acc[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) acc[c] = mk(0.f, 0.f);
    sap_hop<0>(rho_s, lk_s, t, l0, acc);
    sap_hop<1>(rho_s, lk_s, t, l1, acc);
    sap_hop<2>(rho_s, lk_s, t, l2, acc);
    sap_hop<3>(rho_s, lk_s, t, l3, acc);
    cx<float> v[12];
    herm6_mul<float>(cl, rho, v);
    herm6_mul<float>(cl + 36, rho + 6, v + 6);
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
    __syncthreads();  // red_s is read before the next step writes it
  }
  if (XZERO) {
    sp_store(xp, Ve, h, e);
  } else {
#pragma unroll
    for (int c = 0; c < 12; ++c) xs[c] = xs[c] + e[c];
    sp_store(xp, Ve, h, xs);
  }
}

enum { W_SAP_XO = 13 };  // workspace role (free in the solvers' table): odd half of the SAP iterate

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
  if (!xo) return QXD_ENOMEM;
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
      if (cy == 0 && colour == 0)
        hipLaunchKernelGGL(k_sap_half<true>, grid, blk, 0, s, h->geo, sb, colour, nmr, in_e, out_e, xo, V32, He,
                           Ho);
      else
        hipLaunchKernelGGL(k_sap_half<false>, grid, blk, 0, s, h->geo, sb, colour, nmr, in_e, out_e, xo, V32, He,
                           Ho);
    }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_sap_apply(qxd_handle* h, int ncy, int nmr, void* out_e, const void* in_e, void* stream) {
  if (!h || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  return sap_apply_internal(h, ncy, nmr, (float4*)out_e, (const float4*)in_e, as_stream(stream));
}
