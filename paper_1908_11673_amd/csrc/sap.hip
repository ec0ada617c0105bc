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
// Block solver.  The paper's SAP solves the blocks by minimal-residual steps
// on the block's even-odd Schur complement D_hat_B = H_ee - D_eo H_oo^-1 D_oe,
// from the source r_e - D_eo H_oo^-1 r_o, and back-substitutes
// e_o = H_oo^-1 (r_o - D_oe e_e) (eo = 1); eo = 0 runs the steps on D_B itself.
//
// Block layout.  The even-odd half fields keep x3 fastest, so the 256 sites of
// a block sit in runs of two consecutive half indices, and a workgroup reading
// them would use a fraction of every cache line it pulls.  SAP therefore works
// on copies in block order: component k of the site in slot t of block B at
// (B * ncomp + k) * 256 + t, blocks numbered colour-major (B = colour * nhalf +
// j, j the workgroup of that colour's launch).  The plain solver keeps the
// local index s = 64 l0 + 16 l1 + 4 l2 + l3 as the slot; the even-odd one sorts
// a block's sites by parity, the site of parity q in slot 128 q + s / 2, so
// that each wavefront holds sites of one parity.  The
// links (36 float2 a site, forward links of both parities), the clover blocks
// (18 float4) and, on odd sites, their inverses are copied once per gauge field
// and flavour; the iterate x and the source eta (6 float4) live in block order
// for the whole application, and only the first and last half cycles touch the
// half fields.
//
// A workgroup of 256 threads owns one block, one thread per site; a site keeps
// its four forward links in registers.  A hop exchange publishes the spinor of
// the sending sites (24.6 kB of LDS for all 256) and, for each direction, the
// backward hop each owes its forward neighbour, (1 + g_mu) U^+ rho as two
// colour vectors (49.2 kB): 74 kB of LDS per block, so two blocks share a CU.
// With eo = 1 the even wavefronts send while the odd ones receive and the other
// way round; senders and receivers touch disjoint slots, so one barrier per
// exchange suffices.  The residual at entry uses the same exchange for the
// in-block part of D x and global loads for the hops that cross the block's
// faces.  The block reductions of the minimal-residual step go through LDS.
#include "blas.hpp"
#include "sap_blocks.hpp"

namespace {

// Block-order copies of the links, the clover blocks and, for EO, the inverses
// on odd sites (one thread per site; CIb holds 128 odd slots a block).
template <bool EO>
__global__ __launch_bounds__(kSapSites) void k_sap_pack(Geo g, SapGeo sb, const float2* __restrict__ V32,
                                                        const float4* __restrict__ He,
                                                        const float4* __restrict__ Ho,
                                                        const float4* __restrict__ Hi, float2* __restrict__ Vb,
                                                        float4* __restrict__ Cb, float4* __restrict__ CIb) {
  const int B = blockIdx.x, colour = B >= sb.nhalf ? 1 : 0;
  int c0, c1, c2, c3;
  sap_block_coords(sb, colour, B - colour * sb.nhalf, c0, c1, c2, c3);
  const int t = threadIdx.x;
  int l0, l1, l2, l3;
  sap_local<EO>(t, l0, l1, l2, l3);
  const int x0 = kSapB * c0 + l0, x1 = kSapB * c1 + l1, x2 = kSapB * c2 + l2, x3 = kSapB * c3 + l3;
  const int p = (x0 + x1 + x2 + x3) & 1;
  const size_t Ve = g.Ve, h = geo_half(g, x0, x1, x2, x3);
  const float2* Vp = V32 + (size_t)p * 36 * Ve;
  const float4* Hp = p ? Ho : He;
  float2* vb = sap_blk<36>(Vb, B);
  float4* cb = sap_blk<18>(Cb, B);
#pragma unroll 4
  for (int k = 0; k < 36; ++k) vb[k * kSapSites + t] = Vp[(size_t)(k / 9) * 9 * Ve + lk32_index(Ve, k % 9, h)];
#pragma unroll 6
  for (int k = 0; k < 18; ++k) cb[k * kSapSites + t] = Hp[k * Ve + h];
  if (EO && p) {
    float4* ci = CIb + (size_t)B * 18 * (kSapSites / 2) + (t - kSapSites / 2);
#pragma unroll 6
    for (int k = 0; k < 18; ++k) ci[k * (kSapSites / 2)] = Hi[k * Ve + h];
  }
}

// The hop along MU that leaves the block at site x (local coordinate l along
// MU): forward from the face l = 3 with the site's own link u, backward from
// the face l = 0 with the neighbour's link; the neighbour's x in block order.
template <int MU, bool EO>
__device__ __forceinline__ void sap_face(const Geo& g, const SapGeo& sb, int x0, int x1, int x2, int x3, int l,
                                         const float4* __restrict__ Xb, const float2* __restrict__ Vb,
                                         const cx<float> u[9], cx<float> acc[12]) {
  bool neg;
  cx<float> s[12];
  if (l == kSapB - 1) {
    geo_step<MU, +1>(g, x0, x1, x2, x3, neg);
    const int bs = sap_bsite<EO>(sb, x0, x1, x2, x3);
    sp_load(sap_blk<6>(Xb, bs >> 8), kSapSites, bs & 255, s);
    sap_hop_term<MU, true>(acc, s, u, neg);
  } else if (l == 0) {
    geo_step<MU, -1>(g, x0, x1, x2, x3, neg);
    const int bs = sap_bsite<EO>(sb, x0, x1, x2, x3);
    sp_load(sap_blk<6>(Xb, bs >> 8), kSapSites, bs & 255, s);
    cx<float> v[9];
    const float2* vb = sap_blk<36>(Vb, bs >> 8) + MU * 9 * kSapSites + (bs & 255);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      float2 w = vb[k * kSapSites];
      v[k] = mk(w.x, w.y);
    }
    sap_hop_term<MU, false>(acc, s, v, neg);
  }
}

// Block sums of (v, rho) and (v, v) over the workgroup (one barrier).
__device__ __forceinline__ cx<float> sap_alpha(SapLds& L, int t, const cx<float> v[12], const cx<float> rho[12]) {
  float are = 0.f, aim = 0.f, nn = 0.f;
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    are = fmaf(v[c].re, rho[c].re, are);  // conj(v) rho
    are = fmaf(v[c].im, rho[c].im, are);
    aim = fmaf(v[c].re, rho[c].im, aim);
    aim = fmaf(-v[c].im, rho[c].re, aim);
    nn = fmaf(v[c].re, v[c].re, nn);
    nn = fmaf(v[c].im, v[c].im, nn);
  }
  are = sap_wave_sum(are);
  aim = sap_wave_sum(aim);
  nn = sap_wave_sum(nn);
  const int wave = t >> 6;
  if ((t & 63) == 0) {
    L.red[0][wave] = are;
    L.red[1][wave] = aim;
    L.red[2][wave] = nn;
  }
  __syncthreads();
  are = aim = nn = 0.f;
#pragma unroll
  for (int k = 0; k < kSapSites / 64; ++k) {
    are += L.red[0][k];
    aim += L.red[1][k];
    nn += L.red[2][k];
  }
  // alpha = (v, rho) / (v, v); a block whose residual vanished stays put
  return nn > 0.f ? mk(are / nn, aim / nn) : mk(0.f, 0.f);
}

enum { SAP_FIRST = 0, SAP_MID = 1, SAP_LAST = 2 };

// One half cycle on the blocks of `colour` (j = blockIdx.x; its partner is block
// j of the other colour, the other block of the pair {2 k3, 2 k3 + 1} along x3).
//   SAP_FIRST: x = 0 on entry, so r = eta, read from the even half field eta_e
//              (and the odd half eta_o when given, else eta is zero there);
//              also writes the block-order eta of the block and of its partner
//              and zeroes the partner's x;
//   SAP_MID:   r = eta - D x from the block-order fields;
//   SAP_LAST:  as SAP_MID, then writes the block's x and its partner's (final
//              after this half cycle) to out_e on even sites and, when given,
//              to out_o on odd sites.
// EO: even-odd preconditioned block solves (waves 0, 1 hold the even sites).
template <int MODE, bool EO>
__global__ __launch_bounds__(kSapSites, 2) void k_sap_half(Geo g, SapGeo sb, int colour, int nmr,
                                                           const float4* __restrict__ eta_e,
                                                           float4* __restrict__ Eb, float4* __restrict__ Xb,
                                                           const float2* __restrict__ Vb,
                                                           const float4* __restrict__ Cb,
                                                           const float4* __restrict__ CIb,
                                                           float4* __restrict__ out_e,
                                                           const float4* __restrict__ eta_o,
                                                           float4* __restrict__ out_o) {
  __shared__ SapLds L;
  const int j = blockIdx.x;
  int c0, c1, c2, c3;
  sap_block_coords(sb, colour, j, c0, c1, c2, c3);
  const int B = colour * sb.nhalf + j, Bp = (1 - colour) * sb.nhalf + j;
  const SapSite w = sap_site<EO>();
  const int t = w.t, q = w.q;  // q: the site's parity (block origins are even)
  const int x0 = kSapB * c0 + w.l0, x1 = kSapB * c1 + w.l1, x2 = kSapB * c2 + w.l2, x3 = kSapB * c3 + w.l3;
  // the partner's site in the same slot (same parity: x3 moves by 4)
  const int x3p = x3 + ((c3 & 1) ? -kSapB : kSapB);
  const size_t Ve = g.Ve;
  const float4* cb = sap_blk<18>(Cb, B) + t;
  const float4* ci = CIb + (size_t)B * 18 * (kSapSites / 2) + (t - kSapSites / 2);  // odd slots only
  float4* xb = sap_blk<6>(Xb, B);
  float4* eb = sap_blk<6>(Eb, B);

  // the site's four forward links stay in registers for the whole solve
  cx<float> U[4][9];
  {
    const float2* vb = sap_blk<36>(Vb, B) + t;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu)
#pragma unroll
      for (int k = 0; k < 9; ++k) {
        float2 v = vb[(mu * 9 + k) * kSapSites];
        U[mu][k] = mk(v.x, v.y);
      }
  }
  cx<float> rho[12];
  if (MODE == SAP_FIRST) {
    if (q == 0 || eta_o) {
      const float4* src = q ? eta_o : eta_e;
      sp_load(src, Ve, geo_half(g, x0, x1, x2, x3), rho);
      sp_store(eb, kSapSites, t, rho);
      cx<float> ep[12];
      sp_load(src, Ve, geo_half(g, x0, x1, x2, x3p), ep);
      sp_store(sap_blk<6>(Eb, Bp), kSapSites, t, ep);
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = mk(0.f, 0.f);
    }
    cx<float> z[12];
#pragma unroll
    for (int c = 0; c < 12; ++c) z[c] = mk(0.f, 0.f);
    sp_store(sap_blk<6>(Xb, Bp), kSapSites, t, z);
  } else {
    // r = eta - D x = eta - H x + (1/2) (in-block hops + hops across the faces)
    cx<float> xs[12], acc[12];
    sp_load(xb, kSapSites, t, xs);
    sap_publish<EO>(L, xs, U);
    __syncthreads();
    sap_gather<EO>(L, U, acc);
    sap_face<0, EO>(g, sb, x0, x1, x2, x3, w.l0, Xb, Vb, U[0], acc);
    sap_face<1, EO>(g, sb, x0, x1, x2, x3, w.l1, Xb, Vb, U[1], acc);
    sap_face<2, EO>(g, sb, x0, x1, x2, x3, w.l2, Xb, Vb, U[2], acc);
    sap_face<3, EO>(g, sb, x0, x1, x2, x3, w.l3, Xb, Vb, U[3], acc);
    cx<float> hx[12];
    sap_clover<kSapSites>(cb, xs, hx);
    if (q == 0 || eta_o) {
      sp_load(eb, kSapSites, t, rho);
    } else {
#pragma unroll
      for (int c = 0; c < 12; ++c) rho[c] = mk(0.f, 0.f);
    }
#pragma unroll
    for (int c = 0; c < 12; ++c) rho[c] = rho[c] - (hx[c] - 0.5f * acc[c]);
    __syncthreads();  // the exchange buffers are published again below
  }

  // e: the block solution; with EO the odd sites keep r_o in it until the
  // back substitution
  cx<float> e[12];
  if (!EO) {
#pragma unroll
    for (int c = 0; c < 12; ++c) e[c] = mk(0.f, 0.f);
    for (int step = 0; step < nmr; ++step) {
      // v = D_B rho = H rho - (1/2) (in-block hops); every read of the previous
      // step's exchange buffers came before its reduction barrier
      cx<float> acc[12], v[12];
      sap_publish<EO>(L, rho, U);
      __syncthreads();
      sap_gather<EO>(L, U, acc);
      sap_clover<kSapSites>(cb, rho, v);
#pragma unroll
      for (int c = 0; c < 12; ++c) v[c] = v[c] - 0.5f * acc[c];
      const cx<float> alpha = sap_alpha(L, t, v, rho);
#pragma unroll
      for (int c = 0; c < 12; ++c) {
        sap_cmac(e[c], alpha, rho[c]);
        sap_cmac(rho[c], -alpha, v[c]);
      }
    }
  } else {
    // Sends and receives of one exchange touch the slots of opposite parities,
    // so a wave may publish right after it gathered.
#pragma unroll
    for (int c = 0; c < 12; ++c) e[c] = q ? rho[c] : mk(0.f, 0.f);
    if (MODE != SAP_FIRST || eta_o) {
      // source of the Schur system: r_e - D_eo H_oo^-1 r_o = r_e + (1/2) hops(H_oo^-1 r_o)
      if (q == 1) {
        cx<float> so[12];
        sap_clover<kSapSites / 2>(ci, rho, so);
        sap_publish<EO>(L, so, U);
      }
      __syncthreads();
      if (q == 0) {
        cx<float> acc[12];
        sap_gather<EO>(L, U, acc);
#pragma unroll
        for (int c = 0; c < 12; ++c) rho[c] = rho[c] + 0.5f * acc[c];
      }
    }
    for (int step = 0; step < nmr; ++step) {
      // v = D_hat_B rho = H_ee rho + (1/2) hops(t_o), t_o = -(1/2) H_oo^-1 hops(rho)
      if (q == 0) sap_publish<EO>(L, rho, U);
      __syncthreads();
      if (q == 1) {
        cx<float> acc[12], to[12];
        sap_gather<EO>(L, U, acc);
#pragma unroll
        for (int c = 0; c < 12; ++c) acc[c] = -0.5f * acc[c];
        sap_clover<kSapSites / 2>(ci, acc, to);
        sap_publish<EO>(L, to, U);
      }
      __syncthreads();
      cx<float> v[12];
      if (q == 0) {
        cx<float> acc[12];
        sap_gather<EO>(L, U, acc);
        sap_clover<kSapSites>(cb, rho, v);
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = v[c] + 0.5f * acc[c];
      } else {
#pragma unroll
        for (int c = 0; c < 12; ++c) v[c] = mk(0.f, 0.f);
      }
      const cx<float> alpha = sap_alpha(L, t, v, rho);
      if (q == 0) {
#pragma unroll
        for (int c = 0; c < 12; ++c) {
          sap_cmac(e[c], alpha, rho[c]);
          sap_cmac(rho[c], -alpha, v[c]);
        }
      }
    }
    // back substitution: e_o = H_oo^-1 (r_o - D_oe e_e) = H_oo^-1 (r_o + (1/2) hops(e_e))
    if (q == 0) sap_publish<EO>(L, e, U);
    __syncthreads();
    if (q == 1) {
      cx<float> acc[12];
      sap_gather<EO>(L, U, acc);
#pragma unroll
      for (int c = 0; c < 12; ++c) acc[c] = e[c] + 0.5f * acc[c];
      sap_clover<kSapSites / 2>(ci, acc, e);
    }
  }
  if (MODE != SAP_FIRST) {
    cx<float> xs[12];
    sp_load(xb, kSapSites, t, xs);
#pragma unroll
    for (int c = 0; c < 12; ++c) e[c] = e[c] + xs[c];
  }
  sp_store(xb, kSapSites, t, e);
  if (MODE == SAP_LAST && (q == 0 || out_o)) {
    float4* dst = q ? out_o : out_e;
    sp_store(dst, Ve, geo_half(g, x0, x1, x2, x3), e);
    cx<float> xp[12];
    sp_load(sap_blk<6>(Xb, Bp), kSapSites, t, xp);
    sp_store(dst, Ve, geo_half(g, x0, x1, x2, x3p), xp);
  }
}

// workspace roles (free in the solvers' table): block-order links, clover
// blocks, iterate, source and odd-site clover inverses
enum { W_SAP_VB = 8, W_SAP_CB = 9, W_SAP_XB = 13, W_SAP_EB = 14, W_SAP_CIB = 15 };

struct SapArgs {
  Geo g;
  SapGeo sb;
  int nmr;
  const float4* eta_e;
  float4 *Eb, *Xb;
  const float2* Vb;
  const float4 *Cb, *CIb;
  float4* out_e;
  const float4* eta_o;
  float4* out_o;
};

template <int MODE>
void sap_launch(bool eo, const SapArgs& a, int colour, hipStream_t s) {
  const dim3 grid(a.sb.nhalf), blk(kSapSites);
  if (eo)
    hipLaunchKernelGGL((k_sap_half<MODE, true>), grid, blk, 0, s, a.g, a.sb, colour, a.nmr, a.eta_e, a.Eb, a.Xb, a.Vb,
                       a.Cb, a.CIb, a.out_e, a.eta_o, a.out_o);
  else
    hipLaunchKernelGGL((k_sap_half<MODE, false>), grid, blk, 0, s, a.g, a.sb, colour, a.nmr, a.eta_e, a.Eb, a.Xb,
                       a.Vb, a.Cb, a.CIb, a.out_e, a.eta_o, a.out_o);
}

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

namespace {

// The block-order copies of links and clover blocks for slot order eo (made
// when the links, the clover blocks or the slot order changed since the last).
// The inverse blocks on odd sites are copied for the even-odd block solver
// only: the plain one never reads CIb, which then aliases Cb.  The FP32 odd
// clover blocks are cast for the copy and released after it if no other call
// had them, since the block copy holds them from then on (at 128 x 64^3 they
// are 9.7 GB).
qxd_status sap_pack(qxd_handle* h, int eo, float2** Vb, float4** Cb, float4** CIb, SapGeo* sb, hipStream_t s) {
  const size_t V = (size_t)h->V;
  *Vb = (float2*)ws_get(h, W_SAP_VB, V * 36 * sizeof(float2));
  *Cb = (float4*)ws_get(h, W_SAP_CB, V * 18 * sizeof(float4));
  *CIb = eo ? (float4*)ws_get(h, W_SAP_CIB, V / 2 * 18 * sizeof(float4)) : *Cb;
  if (!*Vb || !*Cb || !*CIb) return QXD_ENOMEM;
  const Geo& g = h->geo;
  const int nblk = (g.Le0 / kSapB) * (g.Le1 / kSapB) * (g.Le2 / kSapB) * (g.Le3 / kSapB);
  *sb = SapGeo{g.Le1 / kSapB, g.Le2 / kSapB, g.Le3 / kSapB, nblk / 2};
  // the copies are tagged 2 setup_gen + eo
  const uint64_t tag = 2 * h->setup_gen + (uint64_t)eo;
  if (h->sap_gen != tag) {
    const bool had_ho = (h->copies & CP_HO32) != 0;
    QXD_TRY(ensure_copies(h, CP_V32 | CP_HE32 | CP_HO32 | (eo ? CP_HI32 : 0u), s));
    auto pack = eo ? k_sap_pack<true> : k_sap_pack<false>;
    hipLaunchKernelGGL(pack, dim3(nblk), dim3(kSapSites), 0, s, g, *sb, reinterpret_cast<const float2*>(h->V32),
                       reinterpret_cast<const float4*>(h->He32), reinterpret_cast<const float4*>(h->Ho32),
                       reinterpret_cast<const float4*>(eo ? h->Hi32 : h->Ho32), *Vb, *Cb, *CIb);
    QXD_HIP(hipGetLastError());
    if (!had_ho) {
      QXD_HIP(hipStreamSynchronize(s));
      release_copies(h, CP_HO32);
    }
    h->sap_gen = tag;
  }
  return QXD_OK;
}

}  // namespace

qxd_status sap_blocks(qxd_handle* h, int eo, const float2** Vb, const float4** Cb, SapGeo* sb, hipStream_t s) {
  if (!h->has_inverse) return QXD_ESTATE;
  if (!sap_supported(h)) return QXD_EGEOM;
  float2* vb;
  float4 *cb, *cib;
  QXD_TRY(sap_pack(h, eo, &vb, &cb, &cib, sb, s));
  *Vb = vb;
  *Cb = cb;
  return QXD_OK;
}

qxd_status sap_apply_internal(qxd_handle* h, int ncy, int nmr, int eo, float4* out_e, const float4* in_e,
                              hipStream_t s, const float4* in_o, float4* out_o) {
  if (ncy < 1 || nmr < 1 || ncy > 64 || nmr > 64 || (eo != 0 && eo != 1)) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  if (!sap_supported(h)) return QXD_EGEOM;
  const size_t V = (size_t)h->V;
  float2* Vb;
  float4 *Cb, *CIb;
  SapGeo sb;
  QXD_TRY(sap_pack(h, eo, &Vb, &Cb, &CIb, &sb, s));
  float4* Xb = (float4*)ws_get(h, W_SAP_XB, V * 6 * sizeof(float4));
  float4* Eb = (float4*)ws_get(h, W_SAP_EB, V * 6 * sizeof(float4));
  if (!Xb || !Eb) return QXD_ENOMEM;
  const Geo& g = h->geo;
  const SapArgs a{g, sb, nmr, in_e, Eb, Xb, Vb, Cb, CIb, out_e, in_o, out_o};
  for (int cy = 0; cy < ncy; ++cy)
    for (int colour = 0; colour < 2; ++colour) {
      if (cy == 0 && colour == 0)
        sap_launch<SAP_FIRST>(eo, a, colour, s);
      else if (cy == ncy - 1 && colour == 1)
        sap_launch<SAP_LAST>(eo, a, colour, s);
      else
        sap_launch<SAP_MID>(eo, a, colour, s);
    }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_sap_apply(qxd_handle* h, int ncy, int nmr, int eo, void* out_e, const void* in_e,
                                    void* stream) {
  if (!h || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  return sap_apply_internal(h, ncy, nmr, eo, (float4*)out_e, (const float4*)in_e, as_stream(stream));
}

extern "C" qxd_status qxd_sap_apply_full(qxd_handle* h, int ncy, int nmr, int eo, void* out, const void* in,
                                         void* stream) {
  if (!h || !out || !in || out == in) return QXD_EINVAL;
  const size_t half = (size_t)6 * h->Ve;
  return sap_apply_internal(h, ncy, nmr, eo, (float4*)out, (const float4*)in, as_stream(stream),
                            (const float4*)in + half, (float4*)out + half);
}
