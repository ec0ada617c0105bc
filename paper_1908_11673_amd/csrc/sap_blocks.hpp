// The 4^4 blocks of the Schwarz alternating procedure and of deflation:
// block geometry and block order, and the in-block hop exchange through LDS
// (see sap.hip for the method and the layout).
#pragma once
#include "wilson_site.hpp"

struct SapGeo {
  int nb1, nb2, nb3;  // blocks along x1, x2, x3 (nb3 even)
  int nhalf;          // blocks of one colour
};

namespace {

constexpr int kSapB = 4;                            // block extent
constexpr int kSapSites = kSapB * kSapB * kSapB * kSapB;  // 256: one thread per site


// Slot of the site with local index s and its inverse: parity-sorted for the
// even-odd block solver (EO), the local index itself for the plain one.
template <bool EO>
__device__ __forceinline__ int sap_slot(int s) {
  if (!EO) return s;
  const int q = ((s >> 6) ^ (s >> 4) ^ (s >> 2) ^ s) & 1;
  return (q << 7) | (s >> 1);
}
template <bool EO>
__device__ __forceinline__ void sap_local(int t, int& l0, int& l1, int& l2, int& l3) {
  if (!EO) {
    l0 = t >> 6;
    l1 = (t >> 4) & 3;
    l2 = (t >> 2) & 3;
    l3 = t & 3;
    return;
  }
  const int q = t >> 7, k = t & 127;
  l0 = k >> 5;
  l1 = (k >> 3) & 3;
  l2 = (k >> 1) & 3;
  l3 = 2 * (k & 1) + ((l0 + l1 + l2 + q) & 1);
}

// Block-order index B * 256 + slot of the site x.
template <bool EO>
__device__ __forceinline__ int sap_bsite(const SapGeo& sb, int x0, int x1, int x2, int x3) {
  const int c0 = x0 >> 2, c1 = x1 >> 2, c2 = x2 >> 2, c3 = x3 >> 2;
  const int j = ((c0 * sb.nb1 + c1) * sb.nb2 + c2) * (sb.nb3 >> 1) + (c3 >> 1);
  const int B = ((c0 + c1 + c2 + c3) & 1) * sb.nhalf + j;
  return B * kSapSites + sap_slot<EO>(((x0 & 3) << 6) | ((x1 & 3) << 4) | ((x2 & 3) << 2) | (x3 & 3));
}

// Coordinates of block j of the given colour: along x3 the colours alternate.
__device__ __forceinline__ void sap_block_coords(const SapGeo& sb, int colour, int j, int& c0, int& c1, int& c2,
                                                 int& c3) {
  const int half3 = sb.nb3 >> 1;
  const int k3 = j % half3;
  int line = j / half3;
  c2 = line % sb.nb2;
  line /= sb.nb2;
  c1 = line % sb.nb1;
  c0 = line / sb.nb1;
  c3 = 2 * k3 + ((c0 + c1 + c2 + colour) & 1);
}

template <int NC, class T>
__device__ __forceinline__ T* sap_blk(T* base, int B) {
  return base + (size_t)B * NC * kSapSites;
}

// FP32 arithmetic of the block solver written as fused multiply-adds.  The
// solver is bound by vector instruction issue; a complex multiply-accumulate
// as four FMAs takes 4 instructions where the product-then-sum form takes 6.
// acc += a b
__device__ __forceinline__ void sap_cmac(cx<float>& acc, cx<float> a, cx<float> b) {
  acc.re = fmaf(a.re, b.re, acc.re);
  acc.re = fmaf(-a.im, b.im, acc.re);
  acc.im = fmaf(a.re, b.im, acc.im);
  acc.im = fmaf(a.im, b.re, acc.im);
}
// acc += conj(a) b
__device__ __forceinline__ void sap_cmac_conj(cx<float>& acc, cx<float> a, cx<float> b) {
  acc.re = fmaf(a.re, b.re, acc.re);
  acc.re = fmaf(a.im, b.im, acc.re);
  acc.im = fmaf(a.re, b.im, acc.im);
  acc.im = fmaf(-a.im, b.re, acc.im);
}

// w = u h (FWD) or u^+ h on both colour vectors of a two-spinor
template <bool FWD>
__device__ __forceinline__ void sap_colour_mul(const cx<float> u[9], const cx<float> h0[3], const cx<float> h1[3],
                                               cx<float> w0[3], cx<float> w1[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    w0[a] = mk(0.f, 0.f);
    w1[a] = mk(0.f, 0.f);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      if (FWD) {
        sap_cmac(w0[a], u[3 * a + b], h0[b]);
        sap_cmac(w1[a], u[3 * a + b], h1[b]);
      } else {
        sap_cmac_conj(w0[a], u[3 * b + a], h0[b]);
        sap_cmac_conj(w1[a], u[3 * b + a], h1[b]);
      }
    }
  }
}

// acc += (1 - g_MU) u s (FWD) or (1 + g_MU) u^+ s; neg flips the sign
template <int MU, bool FWD>
__device__ __forceinline__ void sap_hop_term(cx<float> acc[12], const cx<float> s[12], const cx<float> u[9],
                                             bool neg) {
  cx<float> h0[3], h1[3];
  spin_project<MU, FWD>(s, h0, h1);
  if (MU == 0 && neg) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      h0[a] = -h0[a];
      h1[a] = -h1[a];
    }
  }
  cx<float> w0[3], w1[3];
  sap_colour_mul<FWD>(u, h0, h1, w0, w1);
  spin_rebuild_add<MU, FWD>(acc, w0, w1);
}

// out[0..5] = H in[0..5] for one packed Hermitian 6 x 6 block b (36 reals:
// the diagonal, then the entries (i, j), i < j, row by row)
__device__ __forceinline__ void sap_herm6(const float* b, const cx<float>* in, cx<float>* out) {
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = b[i] * in[i];
  int k = 6;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      const cx<float> hij = mk(b[k], b[k + 1]);
      k += 2;
      sap_cmac(out[i], hij, in[j]);
      sap_cmac_conj(out[j], hij, in[i]);
    }
  }
}

// Plain (cached) loads: every step of a block solve reads the clover blocks
// again.  cb points at the site's first component, components STRIDE apart.
template <int STRIDE>
__device__ __forceinline__ void sap_clover(const float4* __restrict__ cb, const cx<float> in[12],
                                           cx<float> out[12]) {
#pragma unroll
  for (int half = 0; half < 2; ++half) {  // one 6 x 6 block at a time: 36 registers of clover
    float r[36];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float4 v = cb[(9 * half + k) * STRIDE];
      r[4 * k] = v.x;
      r[4 * k + 1] = v.y;
      r[4 * k + 2] = v.z;
      r[4 * k + 3] = v.w;
    }
    sap_herm6(r, in + 6 * half, out + 6 * half);
  }
}

// The backward hop that site t contributes to its forward neighbour along MU:
// (1 + g_MU) U(t, MU)^+ rho(t), kept as the two multiplied colour vectors.
template <int MU>
__device__ __forceinline__ void sap_send(float2 (*bw_s)[6][kSapSites], int t, const cx<float> rho[12],
                                         const cx<float> u[9]) {
  cx<float> h0[3], h1[3], w0[3], w1[3];
  spin_project<MU, false>(rho, h0, h1);
  sap_colour_mul<false>(u, h0, h1, w0, w1);
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    bw_s[MU][a][t] = make_float2(w0[a].re, w0[a].im);
    bw_s[MU][3 + a][t] = make_float2(w1[a].re, w1[a].im);
  }
}

// Both in-block hops along MU at the site with local index s and parity q
// (local coordinate l along MU; local-index strides 64, 16, 4, 1): forward with
// the site's own link and the neighbour's rho, backward as sent by the
// neighbour.  Neighbours have the other parity: with EO, slot 128 (1 - q) + s' / 2.
template <int MU, bool EO>
__device__ __forceinline__ void sap_recv(const float4 (*rho_s)[kSapSites], const float2 (*bw_s)[6][kSapSites], int s,
                                         int q, int l, const cx<float> u[9], cx<float> acc[12]) {
  constexpr int st = MU == 0 ? 64 : MU == 1 ? 16 : MU == 2 ? 4 : 1;
  const int other = EO ? (q ^ 1) << 7 : 0;
  if (l < kSapB - 1) {
    const int tn = EO ? other | ((s + st) >> 1) : s + st;
    cx<float> f[12];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      float4 v = rho_s[j][tn];
      f[2 * j] = mk(v.x, v.y);
      f[2 * j + 1] = mk(v.z, v.w);
    }
    sap_hop_term<MU, true>(acc, f, u, false);
  }
  if (l > 0) {
    const int tn = EO ? other | ((s - st) >> 1) : s - st;
    cx<float> w0[3], w1[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float2 v0 = bw_s[MU][a][tn], v1 = bw_s[MU][3 + a][tn];
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

struct SapLds {
  float4 rho[6][kSapSites];
  float2 bw[4][6][kSapSites];
  float red[3][kSapSites / 64];
};

// Where a thread sits in its block: slot t, local index s, parity q, local
// coordinates l (cheap to recompute from the thread index wherever needed).
struct SapSite {
  int t, s, q, l0, l1, l2, l3;
};
template <bool EO>
__device__ __forceinline__ SapSite sap_site() {
  SapSite w;
  w.t = threadIdx.x;
  sap_local<EO>(w.t, w.l0, w.l1, w.l2, w.l3);
  w.q = (w.l0 + w.l1 + w.l2 + w.l3) & 1;
  w.s = (w.l0 << 6) | (w.l1 << 4) | (w.l2 << 2) | w.l3;
  return w;
}

// Publish f at the site (slot t) and the backward hops it owes its forward
// neighbours.
template <bool EO>
__device__ __forceinline__ void sap_publish(SapLds& L, const cx<float> f[12], const cx<float> (*U)[9]) {
  const SapSite w = sap_site<EO>();
#pragma unroll
  for (int j = 0; j < 6; ++j)
    L.rho[j][w.t] = make_float4(f[2 * j].re, f[2 * j].im, f[2 * j + 1].re, f[2 * j + 1].im);
  if (w.l0 < kSapB - 1) sap_send<0>(L.bw, w.t, f, U[0]);
  if (w.l1 < kSapB - 1) sap_send<1>(L.bw, w.t, f, U[1]);
  if (w.l2 < kSapB - 1) sap_send<2>(L.bw, w.t, f, U[2]);
  if (w.l3 < kSapB - 1) sap_send<3>(L.bw, w.t, f, U[3]);
}

// acc = the in-block hops at the site of what its neighbours published.
template <bool EO>
__device__ __forceinline__ void sap_gather(const SapLds& L, const cx<float> (*U)[9], cx<float> acc[12]) {
  const SapSite w = sap_site<EO>();
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = mk(0.f, 0.f);
  sap_recv<0, EO>(L.rho, L.bw, w.s, w.q, w.l0, U[0], acc);
  sap_recv<1, EO>(L.rho, L.bw, w.s, w.q, w.l1, U[1], acc);
  sap_recv<2, EO>(L.rho, L.bw, w.s, w.q, w.l2, U[2], acc);
  sap_recv<3, EO>(L.rho, L.bw, w.s, w.q, w.l3, U[3], acc);
}

}  // namespace

// Block-order copies of the links and clover blocks (sap.hip), made or reused
// for the slot order eo; the geometry of the blocks.
qxd_status sap_blocks(qxd_handle* h, int eo, const float2** Vb, const float4** Cb, SapGeo* sb, hipStream_t s);
