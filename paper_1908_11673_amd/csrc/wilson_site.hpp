// Site-level pieces of the Wilson-clover operator shared by the Schur kernels
// and the SAP block solver: the spin-projected hop along one direction, the
// hop sum at a site (neighbours from coordinates, C* shift of x1 across the
// k <= cstar boundaries), and the two-block clover multiplication.
//
//   (D psi)(x) = H(x) psi(x) - (1/2) hop(psi)(x),
//   hop(psi)(x) = sum_mu (1 - g_mu) V(x,mu) psi(x+mu) + (1 + g_mu) V(x-mu,mu)^+ psi(x-mu)
// (Sec. 2.3 of arXiv:1908.11673, V = U z^qhat, chiral gamma basis).
#pragma once
#include "qxd_internal.hpp"

// The two pieces of a hop on either side of the colour multiplication:
// project s onto the two-spinor (h0, h1) of (1 - g_MU) (FWD) or (1 + g_MU), and
// add the rebuilt four-spinor of the multiplied two-spinor (w0, w1) to acc.
template <int MU, bool FWD, class T>
__device__ __forceinline__ void spin_project(const cx<T> s[12], cx<T> h0[3], cx<T> h1[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const cx<T> s0 = s[a], s1 = s[3 + a], s2 = s[6 + a], s3 = s[9 + a];
    if (MU == 0) {
      h0[a] = FWD ? s0 + s2 : s0 - s2;
      h1[a] = FWD ? s1 + s3 : s1 - s3;
    } else if (MU == 1) {
      h0[a] = FWD ? s0 + ti(s3) : s0 - ti(s3);
      h1[a] = FWD ? s1 + ti(s2) : s1 - ti(s2);
    } else if (MU == 2) {
      h0[a] = FWD ? s0 + s3 : s0 - s3;
      h1[a] = FWD ? s1 - s2 : s1 + s2;
    } else {
      h0[a] = FWD ? s0 + ti(s2) : s0 - ti(s2);
      h1[a] = FWD ? s1 - ti(s3) : s1 + ti(s3);
    }
  }
}

template <int MU, bool FWD, class T>
__device__ __forceinline__ void spin_rebuild_add(cx<T> acc[12], const cx<T> w0[3], const cx<T> w1[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    acc[a] = acc[a] + w0[a];
    acc[3 + a] = acc[3 + a] + w1[a];
    if (MU == 0) {
      acc[6 + a] = FWD ? acc[6 + a] + w0[a] : acc[6 + a] - w0[a];
      acc[9 + a] = FWD ? acc[9 + a] + w1[a] : acc[9 + a] - w1[a];
    } else if (MU == 1) {
      acc[6 + a] = FWD ? acc[6 + a] - ti(w1[a]) : acc[6 + a] + ti(w1[a]);
      acc[9 + a] = FWD ? acc[9 + a] - ti(w0[a]) : acc[9 + a] + ti(w0[a]);
    } else if (MU == 2) {
      acc[6 + a] = FWD ? acc[6 + a] - w1[a] : acc[6 + a] + w1[a];
      acc[9 + a] = FWD ? acc[9 + a] + w0[a] : acc[9 + a] - w0[a];
    } else {
      acc[6 + a] = FWD ? acc[6 + a] - ti(w0[a]) : acc[6 + a] + ti(w0[a]);
      acc[9 + a] = FWD ? acc[9 + a] + ti(w1[a]) : acc[9 + a] - ti(w1[a]);
    }
  }
}

// w = u h (FWD) or u^+ h on both colour vectors of a two-spinor
template <bool FWD, class T>
__device__ __forceinline__ void colour_mul(const cx<T> u[9], const cx<T> h0[3], const cx<T> h1[3], cx<T> w0[3],
                                           cx<T> w1[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    if (FWD) {
      w0[a] = u[3 * a] * h0[0] + u[3 * a + 1] * h0[1] + u[3 * a + 2] * h0[2];
      w1[a] = u[3 * a] * h1[0] + u[3 * a + 1] * h1[1] + u[3 * a + 2] * h1[2];
    } else {
      w0[a] = cmul_conj(u[a], h0[0]) + cmul_conj(u[3 + a], h0[1]) + cmul_conj(u[6 + a], h0[2]);
      w1[a] = cmul_conj(u[a], h1[0]) + cmul_conj(u[3 + a], h1[1]) + cmul_conj(u[6 + a], h1[2]);
    }
  }
}

// Add (1 - g_MU) W s (FWD) or (1 + g_MU) W^+ s (backward) to acc, W the link u;
// neg flips the sign (antiperiodic time wrap).
template <int MU, bool FWD, class T>
__device__ __forceinline__ void hop_term(cx<T> acc[12], const cx<T> s[12], const cx<T> u[9], bool neg) {
  cx<T> h0[3], h1[3];
  spin_project<MU, FWD>(s, h0, h1);
  if (MU == 0 && neg) {
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      h0[a] = -h0[a];
      h1[a] = -h1[a];
    }
  }
  cx<T> w0[3], w1[3];
  colour_mul<FWD>(u, h0, h1, w0, w1);
  spin_rebuild_add<MU, FWD>(acc, w0, w1);
}

template <class T>
__device__ __forceinline__ void g5_lower(cx<T> s[12]) {
#pragma unroll
  for (int c = 6; c < 12; ++c) s[c] = -s[c];
}

// Both hops along MU for the site (p, h) at coordinates x: links of own parity
// are Vp, of the other parity Vq; the field `in` lives on the other parity.
template <int MU, bool G5IN, class T, class SPT, class LKT>
__device__ __forceinline__ void hop_mu(const Geo& g, int h, int x0, int x1, int x2, int x3,
                                       const SPT* __restrict__ in, const LKT* __restrict__ Vp,
                                       const LKT* __restrict__ Vq, cx<T> acc[12]) {
  const size_t Ve = g.Ve;
  bool negf, negb;
  int hf = geo_nb<MU, +1>(g, x0, x1, x2, x3, negf);
  int hb = geo_nb<MU, -1>(g, x0, x1, x2, x3, negb);
  cx<T> s[12], u[9];
  sp_load(in, Ve, hf, s);
  if (G5IN) g5_lower(s);
  lk_load(Vp, Ve, MU, h, u);
  hop_term<MU, true>(acc, s, u, negf);
  sp_load(in, Ve, hb, s);
  if (G5IN) g5_lower(s);
  lk_load(Vq, Ve, MU, hb, u);
  hop_term<MU, false>(acc, s, u, negb);
}

template <bool G5IN, class T, class SPT, class LKT>
__device__ __forceinline__ void hop_site(const Geo& g, int p, int h, const SPT* __restrict__ in,
                                         const LKT* __restrict__ Vp, const LKT* __restrict__ Vq, cx<T> acc[12]) {
  int x0, x1, x2, x3;
  geo_decode(g, p, h, x0, x1, x2, x3);
#pragma unroll
  for (int c = 0; c < 12; ++c) acc[c] = mk(T(0), T(0));
  hop_mu<0, G5IN, T>(g, h, x0, x1, x2, x3, in, Vp, Vq, acc);
  hop_mu<1, G5IN, T>(g, h, x0, x1, x2, x3, in, Vp, Vq, acc);
  hop_mu<2, G5IN, T>(g, h, x0, x1, x2, x3, in, Vp, Vq, acc);
  hop_mu<3, G5IN, T>(g, h, x0, x1, x2, x3, in, Vp, Vq, acc);
}

template <class T, class CLT>
__device__ __forceinline__ void clover_mul(const CLT* __restrict__ C, size_t Ve, int h, const cx<T> in[12],
                                           cx<T> out[12]) {
  T r[72];
  cl_load(C, Ve, h, r);
  herm6_mul<T>(r, in, out);
  herm6_mul<T>(r + 36, in + 6, out + 6);
}

