// Learned preconditioner: three 3^4-tap convolutions on the extended lattice
// (taps follow the C* neighbour map: x + d is the composition of unit steps in
// directions 0..3), real channels 24 -> 32 -> 32 -> 24, no biases, ReLU after
// layers 1 and 2; M(r) = |r| N(r / |r|) on even half fields.
//
// Each layer is an implicit GEMM  out[site][cout] = sum_{tap, cin} in[site + d][cin] W[tap][cout][cin]
// on bf16 MFMA with FP32 accumulation: a wave owns 64 consecutive sites and all
// 32 output channels (4 x 2 tiles of v_mfma_f32_16x16x32_bf16 per tap); each
// lane gathers the 8 input channels it feeds to the matrix core with one
// 16-byte load from the neighbour's channel vector.  Activations are stored as
// [site][32] bf16 (layer-1 input and layer-3 output padded from 24 channels);
// sites are numbered parity-major (even half first), so layer 3 runs on the
// even sites only and writes the spinor layout directly.
//
// Training: the data gradient of a convolution is the convolution with the
// transposed weights on the reversed taps (x + d = z  <=>  x = z - d); the
// weight gradient sum_x g[x][cout] in[x + d][cin] is a GEMM over sites, computed
// on v_mfma_f32_32x32x16_bf16 from tiles transposed through LDS, with per-chunk
// partial sums reduced in a fixed order.  FP32 master weights, Adam.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "blas.hpp"

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f16v __attribute__((ext_vector_type(16)));

#define NN_C 32
#define NN_TAPS 81
#define NN_LAYER_W (NN_TAPS * NN_C * NN_C)  // padded bf16 weights per layer

static const int kCin[3] = {24, 32, 32};
static const int kCout[3] = {32, 32, 24};
static const int kOff[3] = {0, 81 * 32 * 24, 81 * 32 * 24 + 81 * 32 * 32};

struct qxd_nn {
  qxd_handle* h = nullptr;
  float* w = nullptr;      // FP32 master weights (packed as in the header)
  uint16_t* wf = nullptr;  // bf16 forward weights [3][81][32 cout][32 cin]
  uint16_t* wa = nullptr;  // bf16 adjoint weights [3][81 reversed][32 cin][32 cout]
  float *m = nullptr, *v = nullptr, *grad = nullptr;
  int64_t t = 0;
  float skip = 0.f;        // M(r) = |r| (N(rhat) + skip rhat)
  uint16_t *a0 = nullptr, *a1 = nullptr, *a2 = nullptr;  // [V][32]
  uint16_t *g3 = nullptr, *gA = nullptr, *gB = nullptr;  // training: [V][32]
  float* y = nullptr;      // training: raw network output (even half field, F32)
  float *dv = nullptr, *dz = nullptr;  // training, residual loss: D_hat u and D_hat^+ D_hat u
  float* part = nullptr;   // weight-gradient partials
  int nchunk = 0;
  bool blk = false;        // block-tiled convolutions (else per-site gathers)
  int ncu = 1;             // compute units: workgroups of the persistent convolution
};

static const int kWgChunk = 2048;  // sites per weight-gradient workgroup

__device__ inline uint16_t f2bf(float f) { return (uint16_t)f32_to_bf16_bits(f); }
__device__ inline float bf2f(uint16_t b) { return bf16_bits_to_f32(b); }

// unit step of coordinates along mu (C* shift of x1 across the k <= cstar boundaries)
__device__ inline void nn_step(const Geo& g, int* x, int mu, int dir) {
  int Le = mu == 0 ? g.Le0 : mu == 1 ? g.Le1 : mu == 2 ? g.Le2 : g.Le3;
  int v = x[mu] + dir;
  if (v < 0 || v >= Le) {
    v = v < 0 ? v + Le : v - Le;
    if (mu >= 2 && mu <= g.cstar) x[1] = geo_mirror_x1(g, x[1]);
  }
  x[mu] = v;
}

__device__ inline int nn_index(const Geo& g, const int* x) {
  int p = (x[0] + x[1] + x[2] + x[3]) & 1;
  return p * g.Ve + geo_half(g, x[0], x[1], x[2], x[3]);
}

__device__ inline void nn_coords(const Geo& g, int q, int* x) {
  int p = q >= g.Ve ? 1 : 0;
  geo_decode(g, p, q - p * g.Ve, x[0], x[1], x[2], x[3]);
}

__device__ inline bf16x8 ld8(const uint16_t* p) { return *reinterpret_cast<const bf16x8*>(p); }

enum { EPI_RELU = 0, EPI_SPINOR = 1, EPI_MASK = 2 };

// out sites q in [0, nout); in and W as described above.
// EPI_RELU:   out_act[q][c] = bf16(max(acc, 0))
// EPI_SPINOR: out_f (F32 even half field) channel c < 24 = acc * scale (scale = sqrt(scal[i_s]) or 1)
// EPI_MASK:   out_act[q][c] = mask[q][c] > 0 ? bf16(acc) : 0
// SPARSE_IN: the input vanishes on odd sites (layer 1): taps landing on odd
// sites are skipped when the whole wave has one parity.
// EPI_SPINOR also adds skip_coef * rin (rin: F32 even half field, may be null),
// with skip_coef = skip when the output is scaled by |r| (scal given), else
// skip / sqrt(scal2[i_s2]) (the input is normalised at the output of training).
template <int EPI, bool SPARSE_IN>
__global__ __launch_bounds__(256) void k_conv(Geo g, const uint16_t* __restrict__ in, const uint16_t* __restrict__ W,
                                              int nout, uint16_t* __restrict__ out_act, float* __restrict__ out_f,
                                              const uint16_t* __restrict__ mask, const double* __restrict__ scal,
                                              int i_s, const float* __restrict__ rin, float skip,
                                              const double* __restrict__ scal2, int i_s2) {
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int qbase = (blockIdx.x * 4 + wave) * 64;
  if (qbase >= nout) return;
  const int lr = l & 15, kc = (l >> 4) * 8;
  int xs[4][4];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb) {
    int q = qbase + rb * 16 + lr;
    if (q >= nout) q = nout - 1;  // rows past the end compute a copy, never stored
    nn_coords(g, q, xs[rb]);
  }
  const bool uni = (qbase + 64 <= g.Ve) || (qbase >= g.Ve);
  const int pw = qbase >= g.Ve ? 1 : 0;
  f4v acc[4][2];
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb) acc[rb][cb] = f4v{0.f, 0.f, 0.f, 0.f};
  int tap = 0;
  for (int d0 = -1; d0 <= 1; ++d0) {
    int y0[4][4];
#pragma unroll
    for (int rb = 0; rb < 4; ++rb) {
      for (int i = 0; i < 4; ++i) y0[rb][i] = xs[rb][i];
      if (d0) nn_step(g, y0[rb], 0, d0);
    }
    for (int d1 = -1; d1 <= 1; ++d1) {
      int y1[4][4];
#pragma unroll
      for (int rb = 0; rb < 4; ++rb) {
        for (int i = 0; i < 4; ++i) y1[rb][i] = y0[rb][i];
        if (d1) nn_step(g, y1[rb], 1, d1);
      }
      for (int d2 = -1; d2 <= 1; ++d2) {
        int y2[4][4];
#pragma unroll
        for (int rb = 0; rb < 4; ++rb) {
          for (int i = 0; i < 4; ++i) y2[rb][i] = y1[rb][i];
          if (d2) nn_step(g, y2[rb], 2, d2);
        }
        for (int d3 = -1; d3 <= 1; ++d3, ++tap) {
          if (SPARSE_IN && uni) {
            int dist = (d0 != 0) + (d1 != 0) + (d2 != 0) + (d3 != 0);
            if (((pw + dist) & 1) != 0) continue;  // every neighbour is odd: zero input
          }
          const uint16_t* wt = W + tap * (NN_C * NN_C);
          bf16x8 b0 = ld8(wt + lr * NN_C + kc);
          bf16x8 b1 = ld8(wt + (16 + lr) * NN_C + kc);
#pragma unroll
          for (int rb = 0; rb < 4; ++rb) {
            int y3[4];
            for (int i = 0; i < 4; ++i) y3[i] = y2[rb][i];
            if (d3) nn_step(g, y3, 3, d3);
            int qn = nn_index(g, y3);
            bf16x8 a = ld8(in + (size_t)qn * NN_C + kc);
            acc[rb][0] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b0, acc[rb][0], 0, 0, 0);
            acc[rb][1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b1, acc[rb][1], 0, 0, 0);
          }
        }
      }
    }
  }
  float scale = 1.0f, skc = 0.0f;
  if (EPI == EPI_SPINOR && scal) scale = (float)sqrt(scal[i_s]);
  if (EPI == EPI_SPINOR && rin) skc = scal2 ? (float)(skip / sqrt(scal2[i_s2])) : skip;
#pragma unroll
  for (int rb = 0; rb < 4; ++rb)
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        int q = qbase + rb * 16 + (l >> 4) * 4 + i;
        int c = cb * 16 + lr;
        if (q >= nout) continue;
        float vv = acc[rb][cb][i];
        if (EPI == EPI_RELU) {
          out_act[(size_t)q * NN_C + c] = f2bf(fmaxf(vv, 0.f));
        } else if (EPI == EPI_MASK) {
          out_act[(size_t)q * NN_C + c] = mask[(size_t)q * NN_C + c] != 0 && bf2f(mask[(size_t)q * NN_C + c]) > 0.f
                                              ? f2bf(vv)
                                              : (uint16_t)0;
        } else {
          if (c < 24) {
            size_t o = ((size_t)(c >> 2) * g.Ve + q) * 4 + (c & 3);
            out_f[o] = rin ? vv * scale + skc * rin[o] : vv * scale;
          }
        }
      }
}

// ---------------------------------------------------------------------------
// Block-tiled convolution.  The lattice is cut into B0 x B1 x B2 x B3 blocks
// of 512 sites (every B even and dividing the extended extent, so the
// block origin is an even site and local parity equals lattice parity).  The
// block and its one-site halo are staged once in LDS, 64 bytes per site, so
// with the 3^4 stencil each activation is fetched from memory about
// (B+2)^4 / B^4 ~ 4 times instead of 81 times.  The halo follows the C*
// neighbour map (a crossing of a k <= cstar boundary moves x1 by L1; two
// crossings cancel).  Rows of one MFMA tile share a parity, so with an input
// that vanishes on odd sites (SPARSE_IN) the taps landing on odd sites are
// skipped for whole waves and odd halo sites are not loaded.  EVEN_OUT
// computes the even sites only (last layer).
//
// LDS layout: halo coordinates h = b + 1 in [0, B + 2); site (h0, h1, h2, h3)
// at byte h0 T0 + h1 T1 + h2 T2 + 64 h3, its four 16-byte channel chunks
// XOR-swizzled by (h3 / 2) mod 4 against bank conflicts (rows of a tile are
// same-parity sites two apart along x3).  The address is linear in h0..h2 and
// the swizzle depends on h3 only, so each lane keeps three row addresses (one
// per d3) and every tap reads its operands at a compile-time offset.
template <int B0_, int B1_, int B2_, int B3_>
struct NnShape {
  static constexpr int B0 = B0_, B1 = B1_, B2 = B2_, B3 = B3_;
  static constexpr int H0 = B0 + 2, H1 = B1 + 2, H2 = B2 + 2, H3 = B3 + 2;
  static constexpr int NPOS = H0 * H1 * H2 * H3;
  static constexpr int T2 = 64 * H3, T1 = T2 * H2, T0 = T1 * H1;
  static constexpr int LDS_BYTES = (NPOS + 127) / 128 * 128 * 64;  // halo rounded up to 128 positions
  static_assert(B0 * B1 * B2 * B3 == 512, "blocks of 512 sites");
  static_assert(B0 % 2 == 0 && B1 % 2 == 0 && B2 % 2 == 0 && B3 % 2 == 0, "even block extents");
  static_assert(LDS_BYTES <= 163840, "halo exceeds the LDS");
  static_assert(2 * (T0 + T1 + T2) < 65536, "tap offsets exceed the LDS immediate");
};

#define NN_BLK_SITES 512
// t x x1 x x2 x x3 extents of the blocks: the x3 extent 8 keeps four
// same-parity sites (256 contiguous bytes of activations) per x3 line
typedef NnShape<4, 4, 4, 8> NnBlock;

// byte address of chunk c of halo site h (see the layout above)
template <class SH>
__device__ __forceinline__ int nn_lds_addr(int h0, int h1, int h2, int h3, int c) {
  return h0 * SH::T0 + h1 * SH::T1 + h2 * SH::T2 + 64 * h3 + ((c ^ ((h3 >> 1) & 3)) << 4);
}

// j-th site of parity p inside the block: local coordinates
template <class SH>
__device__ __forceinline__ void nn_blk_site(int p, int j, int& b0, int& b1, int& b2, int& b3) {
  constexpr int r3 = SH::B3 / 2;
  int k = j % r3, line = j / r3;
  b2 = line % SH::B2;
  line /= SH::B2;
  b1 = line % SH::B1;
  b0 = line / SH::B1;
  b3 = 2 * k + ((b0 + b1 + b2 + p) & 1);
}

// Taps a wave of parity-P rows contracts: all 81, or with an input that
// vanishes on odd sites only those whose neighbours are even (P + |d| even).
template <bool SPARSE, int P>
struct NnTapList {
  int n = 0;
  int t[81] = {};
  constexpr NnTapList() {
    for (int tap = 0; tap < 81; ++tap) {
      int dist = (tap / 27 != 1) + (tap / 9 % 3 != 1) + (tap / 3 % 3 != 1) + (tap % 3 != 1);
      if (!SPARSE || ((P + dist) & 1) == 0) t[n++] = tap;
    }
  }
};

// The tap loop, fully unrolled: the weights of tap k + NN_WPF and the LDS
// operands of tap k + APF are requested while tap k is contracted, on NCB
// column tiles of 16 output channels starting at tile cb0; side(k) issues
// further loads of the caller's (the next block's halo) in tap k.  raddr[rb][d3 + 1] is the byte
// address of row rb's neighbour at (-1, -1, -1, d3); tap (d0, d1, d2, d3)
// adds the constant (d0 + 1) T0 + (d1 + 1) T1 + (d2 + 1) T2.
#ifndef NN_WPF
#define NN_WPF 4  // taps ahead whose weights are in flight
#endif
#ifndef NN_WAVES
#define NN_WAVES 8  // waves per workgroup of the block kernel
#endif
#ifndef NN_APF
#define NN_APF 2  // taps ahead whose LDS operands are in flight
#endif
template <class SH, bool SPARSE, int P, int RB, int NCB, class PF>
__device__ __forceinline__ void nn_blk_taps(const char* lds, const uint16_t* __restrict__ W, const int (&raddr)[RB][3],
                                            int lr, int kc, int cb0, f4v (&acc)[RB][NCB], PF&& side) {
  constexpr NnTapList<SPARSE, P> TL{};
  // LDS operands of APF taps ahead: 8 row tiles hold 32 registers per tap in flight
  constexpr int APF = RB >= 8 ? 1 : NN_APF;
  static_assert(TL.n > NN_WPF && TL.n > APF, "prefetch deeper than the tap list");
  auto wld = [&](int tap, int cb) {
    return ld8(W + tap * (NN_C * NN_C) + ((cb0 + cb) * 16 + lr) * NN_C + kc);
  };
  auto rd = [&](int rb, int tap) {
    const int off = (tap / 27) * SH::T0 + (tap / 9 % 3) * SH::T1 + (tap / 3 % 3) * SH::T2;
    return *reinterpret_cast<const bf16x8*>(lds + raddr[rb][tap % 3] + off);
  };
  bf16x8 wb[NN_WPF][NCB];
#pragma unroll
  for (int k = 0; k < NN_WPF; ++k)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) wb[k][cb] = wld(TL.t[k], cb);
  bf16x8 a[APF + 1][RB];
#pragma unroll
  for (int k = 0; k < APF; ++k)
#pragma unroll
    for (int rb = 0; rb < RB; ++rb) a[k][rb] = rd(rb, TL.t[k]);
  // an explicit count: a plain full-unroll request is dropped above LLVM's
  // size limit, which this loop body with its halo loads exceeds
#pragma unroll TL.n
  for (int k = 0; k < TL.n; ++k) {
    bf16x8 w[NCB];
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) w[cb] = wb[k % NN_WPF][cb];
    if (k + NN_WPF < TL.n) {
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) wb[k % NN_WPF][cb] = wld(TL.t[k + NN_WPF], cb);
    }
    side(k);
    if (k + APF < TL.n) {
#pragma unroll
      for (int rb = 0; rb < RB; ++rb) a[(k + APF) % (APF + 1)][rb] = rd(rb, TL.t[k + APF]);
    }
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb)
        acc[rb][cb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[k % (APF + 1)][rb], w[cb], acc[rb][cb], 0, 0, 0);
    // keep each tap's prefetches in this tap: left free, the scheduler sinks
    // every load next to its first use to save registers, and each tap then
    // waits for its own weights and LDS operands
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Halo of the block with origin o, moved through registers: this thread
// moves chunk threadIdx & 3 of the positions threadIdx / 4 + GRP k, k < HPT.
// Positions past the halo and skipped odd sites read the first site; they
// are written to LDS but never read.
template <class SH, int NW, bool SPARSE_IN>
struct NnHalo {
  static constexpr int GRP = 16 * NW;                     // positions per pass of the workgroup
  static constexpr int HPT = (SH::NPOS + GRP - 1) / GRP;  // positions per thread
  static_assert(HPT * GRP * 64 <= SH::LDS_BYTES, "halo staging");
  __device__ static __forceinline__ uint4 load(const Geo& g, const uint16_t* __restrict__ in, int o0, int o1, int o2,
                                               int o3, int k) {
    int pos = (threadIdx.x >> 2) + GRP * k;
    // opaque: otherwise the block-independent coordinates of all HPT
    // positions are hoisted out of the block loop and held in registers
    asm volatile("" : "+v"(pos));
    bool ok = pos < SH::NPOS;
    int h3 = pos % SH::H3, r = pos / SH::H3;
    int h2 = r % SH::H2;
    r /= SH::H2;
    int h1 = r % SH::H1, h0 = r / SH::H1;
    int x0 = o0 + h0 - 1, x1 = o1 + h1 - 1, x2 = o2 + h2 - 1, x3 = o3 + h3 - 1;
    x0 = x0 < 0 ? x0 + g.Le0 : (x0 >= g.Le0 ? x0 - g.Le0 : x0);
    x1 = x1 < 0 ? x1 + g.Le1 : (x1 >= g.Le1 ? x1 - g.Le1 : x1);
    bool mir = false;
    if (x2 < 0 || x2 >= g.Le2) {
      x2 = x2 < 0 ? x2 + g.Le2 : x2 - g.Le2;
      mir = g.cstar >= 2;
    }
    if (x3 < 0 || x3 >= g.Le3) {
      x3 = x3 < 0 ? x3 + g.Le3 : x3 - g.Le3;
      if (g.cstar >= 3) mir = !mir;
    }
    if (mir) x1 = geo_mirror_x1(g, x1);
    int par = (x0 + x1 + x2 + x3) & 1;
    ok = ok && !(SPARSE_IN && par);
    size_t q = ok ? (size_t)par * g.Ve + geo_half(g, x0, x1, x2, x3) : 0;
    return reinterpret_cast<const uint4*>(in + q * NN_C)[threadIdx.x & 3];
  }
  __device__ static __forceinline__ void store(char* lds, int k, const uint4& v) {
    int pos = (threadIdx.x >> 2) + GRP * k;
    int h3 = pos % SH::H3;
    *reinterpret_cast<uint4*>(lds + pos * 64 + (((threadIdx.x & 3) ^ ((h3 >> 1) & 3)) << 4)) = v;
  }
};

// Persistent block-tiled convolution: a workgroup of NW = 8 waves (two per
// SIMD, one workgroup per CU) walks blocks, and the workgroups of one XCD walk
// one contiguous eighth of the block list together, so neighbouring blocks
// share that XCD's L2.  A wave owns 8 row tiles of 16 same-parity sites (128
// sites) and one column tile of 16 output channels, so each weight tile it
// loads feeds 8 matrix-core instructions (the last layer: 4 tiles of even
// sites).  Each operand read from LDS feeds one instruction: the LDS has the
// bandwidth to spare, the vector memory path that brings the weights has
// not (half the weight loads of a wave owning both column tiles of 4 row
// tiles, for twice the LDS reads).  Per block: taps (with the next block's
// halo loads), output tile staged in LDS, coalesced stores, the next halo
// from registers to LDS.
template <int NW, int EPI, bool SPARSE_IN, bool EVEN_OUT>
__global__ __launch_bounds__(64 * NW) void k_conv_ws(Geo g, int nblk, const uint16_t* __restrict__ in,
                                                 const uint16_t* __restrict__ W, uint16_t* __restrict__ out_act,
                                                 float* __restrict__ out_f, const uint16_t* __restrict__ mask,
                                                 const double* __restrict__ scal, int i_s,
                                                 const float* __restrict__ rin, float skip,
                                                 const double* __restrict__ scal2, int i_s2) {
  using SH = NnBlock;
  __shared__ uint4 lds4[SH::LDS_BYTES / 16];
  char* lds = reinterpret_cast<char*>(lds4);
  const int n1 = g.Le1 / SH::B1, n2 = g.Le2 / SH::B2, n3 = g.Le3 / SH::B3;
  // this workgroup's blocks: group x = blockIdx % nx (the XCD when nx = 8) owns
  // blocks [x per, (x + 1) per), walked by its nwx workgroups in turn
  const int nx = min(8, (int)gridDim.x);
  const int xcd = blockIdx.x % nx, wi = blockIdx.x / nx;
  const int nwx = ((int)gridDim.x - xcd + nx - 1) / nx;
  const int per = (nblk + nx - 1) / nx;
  const int bbeg = min(nblk, xcd * per), bend = min(nblk, (xcd + 1) * per);
  auto origin = [&](int b, int& o0, int& o1, int& o2, int& o3) {
    int c3 = b % n3, t = b / n3;
    int c2 = t % n2;
    t /= n2;
    int c1 = t % n1, c0 = t / n1;
    o0 = c0 * SH::B0;
    o1 = c1 * SH::B1;
    o2 = c2 * SH::B2;
    o3 = c3 * SH::B3;
  };

  // NW waves share the 32 row tiles (16 of each parity) and the two column
  // tiles, each wave one column tile; with EVEN_OUT the 16 even row tiles
  constexpr int NCB = 1;
  constexpr int RB = EVEN_OUT ? 32 / NW : 64 / NW;
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l & 15, kc = (l >> 4) * 8, ch = l >> 4;
  const int p = EVEN_OUT ? 0 : wave / (NW / 2);
  const int cb0 = wave & 1;
  const int g0 = EVEN_OUT ? (wave >> 1) : (wave % (NW / 2)) >> 1, gstep = EVEN_OUT ? NW / 2 : NW / 4;
  int raddr[RB][3];
#pragma unroll
  for (int rb = 0; rb < RB; ++rb) {
    int b0, b1, b2, b3;
    nn_blk_site<SH>(p, (g0 + rb * gstep) * 16 + lr, b0, b1, b2, b3);
#pragma unroll
    for (int d3 = 0; d3 < 3; ++d3) raddr[rb][d3] = nn_lds_addr<SH>(b0, b1, b2, b3 + d3, ch);
  }
  float scale = 1.0f, skc = 0.0f;
  if (EPI == EPI_SPINOR) {
    if (scal) scale = (float)sqrt(scal[i_s]);
    if (rin) skc = scal2 ? (float)(skip / sqrt(scal2[i_s2])) : skip;
  }

  // The halo of the next block is loaded into registers during the taps of
  // the current one (HPT loads per thread, one per tap) and written to the LDS
  // once its output tile has left: the loads of all workgroups then spread
  // over the matrix-core work instead of arriving at memory in one burst per
  // block.
  using HL = NnHalo<SH, NW, SPARSE_IN>;
  // one halo load every HS taps, spread over the tap loop
  constexpr int NTAP0 = NnTapList<SPARSE_IN, 0>{}.n, NTAP1 = NnTapList<SPARSE_IN, 1>{}.n;
  constexpr int HS = (NTAP0 < NTAP1 ? NTAP0 : NTAP1) / HL::HPT;
  static_assert(HS >= 1, "one halo load per tap at most");
  uint4 hv[HL::HPT];
  if (bbeg + wi < bend) {
    int o0, o1, o2, o3;
    origin(bbeg + wi, o0, o1, o2, o3);
#pragma unroll
    for (int k = 0; k < HL::HPT; ++k) hv[k] = HL::load(g, in, o0, o1, o2, o3, k);
#pragma unroll
    for (int k = 0; k < HL::HPT; ++k) HL::store(lds, k, hv[k]);
  }
  __syncthreads();

  for (int b = bbeg + wi; b < bend; b += nwx) {
    int o0, o1, o2, o3;
    origin(b, o0, o1, o2, o3);
    // the next block of this workgroup (the last one loads a block it does not use)
    int n0, n1h, n2h, n3h;
    origin(min(b + nwx, bend - 1), n0, n1h, n2h, n3h);
    auto side = [&](int k) {
      if (k % HS == 0 && k / HS < HL::HPT) hv[k / HS] = HL::load(g, in, n0, n1h, n2h, n3h, k / HS);
    };
    f4v acc[RB][NCB];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) acc[rb][cb] = f4v{0.f, 0.f, 0.f, 0.f};
    // the weight loads do not depend on the block: keep the compiler from
    // hoisting all 81 taps' worth out of the block loop.  The opaque value is
    // an offset, not the pointer: a pointer passed through the asm loses its
    // global address space, and the flat loads the compiler then emits count
    // against the LDS wait counter too, so every wait for an LDS operand
    // would also wait for the weight loads in flight.
    int wofs = 0;
    asm volatile("" : "+s"(wofs));
    const uint16_t* Wb = W + wofs;
    if (!SPARSE_IN || p == 0)
      nn_blk_taps<SH, SPARSE_IN, 0, RB, NCB>(lds, Wb, raddr, lr, kc, cb0, acc, side);
    else
      nn_blk_taps<SH, SPARSE_IN, 1, RB, NCB>(lds, Wb, raddr, lr, kc, cb0, acc, side);
    __syncthreads();  // every wave is done with the halo: the LDS takes the output tile
    const int hb = geo_half(g, o0, o1, o2, o3);
    if (EPI == EPI_SPINOR) {
      // even sites only: tile [256][24] FP32, then float4 stores per (component group, site)
      float* st = reinterpret_cast<float*>(lds);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int j = (g0 + rb * gstep) * 16 + (l >> 4) * 4 + i;
            int c = (cb0 + cb) * 16 + lr;
            if (c < 24) st[j * 24 + c] = acc[rb][cb][i];
          }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < 6 * 4 / NW; ++it) {
        int idx = threadIdx.x + 64 * NW * it;
        int j = idx % (NN_BLK_SITES / 2), slot = idx / (NN_BLK_SITES / 2);
        int b0, b1, b2, b3;
        nn_blk_site<SH>(0, j, b0, b1, b2, b3);
        size_t o = (size_t)slot * g.Ve + hb + geo_half(g, b0, b1, b2, b3);
        float4 v = *reinterpret_cast<const float4*>(st + j * 24 + slot * 4);
        v.x *= scale;
        v.y *= scale;
        v.z *= scale;
        v.w *= scale;
        if (rin) {
          float4 r4 = reinterpret_cast<const float4*>(rin)[o];
          v.x += skc * r4.x;
          v.y += skc * r4.y;
          v.z += skc * r4.z;
          v.w += skc * r4.w;
        }
        reinterpret_cast<float4*>(out_f)[o] = v;
      }
    } else {
      // tile [512][32] bf16 (site s = parity * 256 + j), then 16-byte stores
      uint16_t* st = reinterpret_cast<uint16_t*>(lds);
#pragma unroll
      for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb)
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            int s = p * (NN_BLK_SITES / 2) + (g0 + rb * gstep) * 16 + (l >> 4) * 4 + i;
            float vv = acc[rb][cb][i];
            st[s * NN_C + (cb0 + cb) * 16 + lr] = f2bf(EPI == EPI_RELU ? fmaxf(vv, 0.f) : vv);
          }
      __syncthreads();
#pragma unroll
      for (int it = 0; it < 8 * 4 / NW; ++it) {
        int idx = threadIdx.x + 64 * NW * it;
        int s = idx >> 2, c = idx & 3;
        int ps = s / (NN_BLK_SITES / 2), j = s % (NN_BLK_SITES / 2);
        int b0, b1, b2, b3;
        nn_blk_site<SH>(ps, j, b0, b1, b2, b3);
        size_t q = (size_t)ps * g.Ve + hb + geo_half(g, b0, b1, b2, b3);
        uint4 v = *reinterpret_cast<const uint4*>(st + s * NN_C + c * 8);
        if (EPI == EPI_MASK) {
          uint4 m = *reinterpret_cast<const uint4*>(mask + q * NN_C + c * 8);
          uint32_t* vw = reinterpret_cast<uint32_t*>(&v);
          const uint32_t* mw = reinterpret_cast<const uint32_t*>(&m);
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            uint32_t keep = (bf16lo(mw[k]) > 0.f ? 0x0000ffffu : 0u) | (bf16hi(mw[k]) > 0.f ? 0xffff0000u : 0u);
            vw[k] &= keep;
          }
        }
        *reinterpret_cast<uint4*>(out_act + q * NN_C + c * 8) = v;
      }
    }
    __syncthreads();  // the output tile has left the LDS
    if (b + nwx < bend) {
#pragma unroll
      for (int k = 0; k < HL::HPT; ++k) HL::store(lds, k, hv[k]);
    }
    __syncthreads();
  }
}

// layer-1 input: even sites carry r / |r| (channel 2c + 0/1 = Re/Im of
// component c), odd sites and channels 24..31 are zero.  Only channels 0..23
// of the even sites are written here: the rest of a0 is zeroed once when it
// is allocated and never written.
__global__ __launch_bounds__(256) void k_nn_embed(Geo g, const float4* __restrict__ r, const double* __restrict__ scal,
                                                  int i_n2, uint16_t* __restrict__ a0) {
  int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= g.Ve) return;
  uint16_t v[24];
  float s = scal ? (float)(1.0 / sqrt(scal[i_n2])) : 1.0f;
  for (int j = 0; j < 6; ++j) {
    float4 x = r[(size_t)j * g.Ve + q];
    v[4 * j] = f2bf(s * x.x);
    v[4 * j + 1] = f2bf(s * x.y);
    v[4 * j + 2] = f2bf(s * x.z);
    v[4 * j + 3] = f2bf(s * x.w);
  }
  uint4* o = reinterpret_cast<uint4*>(a0 + (size_t)q * NN_C);
  for (int k = 0; k < 3; ++k)
    o[k] = make_uint4(v[8 * k] | (v[8 * k + 1] << 16), v[8 * k + 2] | (v[8 * k + 3] << 16),
                      v[8 * k + 4] | (v[8 * k + 5] << 16), v[8 * k + 6] | (v[8 * k + 7] << 16));
}

// padded bf16 forward and adjoint weights from the FP32 master copy
__global__ void k_nn_pack(const float* __restrict__ w, uint16_t* __restrict__ wf, uint16_t* __restrict__ wa) {
  int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= 3 * NN_LAYER_W) return;
  int layer = t / NN_LAYER_W, r = t % NN_LAYER_W;
  int tap = r / (NN_C * NN_C), co = (r / NN_C) % NN_C, ci = r % NN_C;
  const int cin = layer == 0 ? 24 : 32, cout = layer == 2 ? 24 : 32;
  const int off = layer == 0 ? 0 : layer == 1 ? 81 * 32 * 24 : 81 * 32 * 24 + 81 * 32 * 32;
  float val = (co < cout && ci < cin) ? w[off + (tap * cout + co) * cin + ci] : 0.f;
  uint16_t b = f2bf(val);
  wf[t] = b;
  // adjoint: reversed tap, transposed channels
  wa[layer * NN_LAYER_W + ((80 - tap) * NN_C + ci) * NN_C + co] = b;
}

// loss of one pair and the gradient at the network output (even sites):
// d = y - e / |r|;  g = 2 d |r|^2 / (|e|^2 B);  partial sum of |d|^2
__global__ __launch_bounds__(256) void k_nn_lossgrad(Geo g, const float4* __restrict__ y, const float4* __restrict__ e,
                                                     const double* __restrict__ scal, int i_r2, int i_e2, double invB,
                                                     uint16_t* __restrict__ g3, double* __restrict__ partial) {
  __shared__ double sh[4];
  int q = blockIdx.x * 256 + threadIdx.x;
  double a = 0.0;
  if (q < g.Ve) {
    double r2 = scal[i_r2], e2 = scal[i_e2];
    float ir = (float)(1.0 / sqrt(r2));
    float f = (float)(2.0 * r2 / e2 * invB);
    uint16_t v[NN_C];
    for (int c = 0; c < NN_C; ++c) v[c] = 0;
    for (int j = 0; j < 6; ++j) {
      float4 yy = y[(size_t)j * g.Ve + q], ee = e[(size_t)j * g.Ve + q];
      float d[4] = {yy.x - ir * ee.x, yy.y - ir * ee.y, yy.z - ir * ee.z, yy.w - ir * ee.w};
      for (int k = 0; k < 4; ++k) {
        a += (double)d[k] * (double)d[k];
        v[4 * j + k] = f2bf(f * d[k]);
      }
    }
    uint4* o = reinterpret_cast<uint4*>(g3 + (size_t)q * NN_C);
    for (int k = 0; k < 4; ++k)
      o[k] = make_uint4(v[8 * k] | (v[8 * k + 1] << 16), v[8 * k + 2] | (v[8 * k + 3] << 16),
                        v[8 * k + 4] | (v[8 * k + 5] << 16), v[8 * k + 6] | (v[8 * k + 7] << 16));
  }
  for (int off = 32; off > 0; off >>= 1) a += __shfl_xor(a, off);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// u = y - e / |r| (in place in y)
__global__ __launch_bounds__(256) void k_nn_err(int Ve, float4* __restrict__ y, const float4* __restrict__ e,
                                                const double* __restrict__ scal, int i_r2) {
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (size_t)6 * Ve) return;
  float ir = (float)(1.0 / sqrt(scal[i_r2]));
  float4 a = y[i], b = e[i];
  y[i] = make_float4(a.x - ir * b.x, a.y - ir * b.y, a.z - ir * b.z, a.w - ir * b.w);
}

// g3 on the even sites = f * z (F32 even half field), channels 24..31 zero
__global__ __launch_bounds__(256) void k_nn_embed_grad(int Ve, const float4* __restrict__ z, float f,
                                                       uint16_t* __restrict__ g3) {
  int q = blockIdx.x * 256 + threadIdx.x;
  if (q >= Ve) return;
  uint16_t v[NN_C];
  for (int c = 0; c < NN_C; ++c) v[c] = 0;
  for (int j = 0; j < 6; ++j) {
    float4 x = z[(size_t)j * Ve + q];
    v[4 * j] = f2bf(f * x.x);
    v[4 * j + 1] = f2bf(f * x.y);
    v[4 * j + 2] = f2bf(f * x.z);
    v[4 * j + 3] = f2bf(f * x.w);
  }
  uint4* o = reinterpret_cast<uint4*>(g3 + (size_t)q * NN_C);
  for (int k = 0; k < 4; ++k)
    o[k] = make_uint4(v[8 * k] | (v[8 * k + 1] << 16), v[8 * k + 2] | (v[8 * k + 3] << 16),
                      v[8 * k + 4] | (v[8 * k + 5] << 16), v[8 * k + 6] | (v[8 * k + 7] << 16));
}

// weight-gradient partials: part[chunk][tap][co][ci] = sum_{q in chunk} gq[q][co] in[q + d][ci]
// block: 4 waves, wave w takes tap blockIdx.y * 4 + w; sites in tiles of 64 transposed through LDS
__global__ __launch_bounds__(256) void k_conv_wgrad(Geo g, const uint16_t* __restrict__ gq,
                                                    const uint16_t* __restrict__ in, int nq, int chunk,
                                                    float* __restrict__ part) {
  __shared__ __attribute__((aligned(16))) uint16_t gT[NN_C][72];
  __shared__ __attribute__((aligned(16))) uint16_t aT[4][NN_C][72];
  const int wave = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int tap = blockIdx.y * 4 + wave;
  const bool tap_ok = tap < NN_TAPS;
  const int d0 = tap / 27 - 1, d1 = (tap / 9) % 3 - 1, d2 = (tap / 3) % 3 - 1, d3 = tap % 3 - 1;
  f16v acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  const int q_begin = blockIdx.x * chunk;
  for (int q0 = q_begin; q0 < q_begin + chunk && q0 < nq; q0 += 64) {
    __syncthreads();
    {
      int si = threadIdx.x >> 2, c8 = (threadIdx.x & 3) * 8;
      int q = q0 + si;
      uint4 v = make_uint4(0, 0, 0, 0);
      if (q < nq) v = *reinterpret_cast<const uint4*>(gq + (size_t)q * NN_C + c8);
      uint32_t w4[4] = {v.x, v.y, v.z, v.w};
      for (int i = 0; i < 4; ++i) {
        gT[c8 + 2 * i][si] = (uint16_t)(w4[i] & 0xffff);
        gT[c8 + 2 * i + 1][si] = (uint16_t)(w4[i] >> 16);
      }
    }
    if (tap_ok) {
      int q = q0 + l;
      bool ok = q < nq;
      int x[4];
      nn_coords(g, ok ? q : 0, x);
      if (d0) nn_step(g, x, 0, d0);
      if (d1) nn_step(g, x, 1, d1);
      if (d2) nn_step(g, x, 2, d2);
      if (d3) nn_step(g, x, 3, d3);
      int qn = nn_index(g, x);
      for (int c8 = 0; c8 < NN_C; c8 += 8) {
        uint4 v = make_uint4(0, 0, 0, 0);
        if (ok) v = *reinterpret_cast<const uint4*>(in + (size_t)qn * NN_C + c8);
        uint32_t w4[4] = {v.x, v.y, v.z, v.w};
        for (int i = 0; i < 4; ++i) {
          aT[wave][c8 + 2 * i][l] = (uint16_t)(w4[i] & 0xffff);
          aT[wave][c8 + 2 * i + 1][l] = (uint16_t)(w4[i] >> 16);
        }
      }
    }
    __syncthreads();
    if (tap_ok) {
#pragma unroll
      for (int k0 = 0; k0 < 64; k0 += 16) {
        int kk = k0 + (l >> 5) * 8;
        bf16x8 a = *reinterpret_cast<const bf16x8*>(&gT[l & 31][kk]);
        bf16x8 b = *reinterpret_cast<const bf16x8*>(&aT[wave][l & 31][kk]);
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, acc, 0, 0, 0);
      }
    }
  }
  if (tap_ok) {
    float* o = part + ((size_t)blockIdx.x * NN_TAPS + tap) * (NN_C * NN_C);
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      int row = (i / 4) * 8 + (l >> 5) * 4 + (i & 3);
      o[row * NN_C + (l & 31)] = acc[i];
    }
  }
}

// grad[off + (tap cout + co) cin + ci] += sum over chunks (fixed order)
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nchunk, int cin, int cout, int off,
                               float* __restrict__ grad) {
  int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= NN_TAPS * cout * cin) return;
  int tap = t / (cout * cin), co = (t / cin) % cout, ci = t % cin;
  double s = 0.0;
  for (int c = 0; c < nchunk; ++c) s += part[((size_t)c * NN_TAPS + tap) * (NN_C * NN_C) + co * NN_C + ci];
  grad[off + t] += (float)s;
}

__global__ void k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2) {
  int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float gi = g[i];
  float mi = b1 * m[i] + (1.f - b1) * gi;
  float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------------------
// host side

static qxd_status nn_repack(qxd_nn* net, hipStream_t s) {
  hipLaunchKernelGGL(k_nn_pack, dim3(div_up(3 * NN_LAYER_W, 256)), dim3(256), 0, s, net->w, net->wf, net->wa);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

static void conv_launch_blk(qxd_handle* h, const qxd_nn* net, int layer, const uint16_t* in, const uint16_t* wl,
                            int epi, uint16_t* out_act, float* out_f, const uint16_t* mask, const double* scal, int i_s,
                            hipStream_t s, const float* rin, float skip, const double* scal2, int i_s2) {
  const int nblk = (int)(h->V / NN_BLK_SITES);
  constexpr int NW = NN_WAVES;
  dim3 grid((unsigned)std::min(nblk, net->ncu)), blk(64 * NW);
  // the layer-1 input and the layer-3 output gradient vanish on odd sites
  if (epi == EPI_RELU && layer == 0)
    hipLaunchKernelGGL((k_conv_ws<NW, EPI_RELU, true, false>), grid, blk, 0, s, h->geo, nblk, in, wl, out_act, out_f, mask,
                       scal, i_s, rin, skip, scal2, i_s2);
  else if (epi == EPI_RELU)
    hipLaunchKernelGGL((k_conv_ws<NW, EPI_RELU, false, false>), grid, blk, 0, s, h->geo, nblk, in, wl, out_act, out_f,
                       mask, scal, i_s, rin, skip, scal2, i_s2);
  else if (epi == EPI_SPINOR)
    hipLaunchKernelGGL((k_conv_ws<NW, EPI_SPINOR, false, true>), grid, blk, 0, s, h->geo, nblk, in, wl, out_act, out_f,
                       mask, scal, i_s, rin, skip, scal2, i_s2);
  else if (layer == 2)
    hipLaunchKernelGGL((k_conv_ws<NW, EPI_MASK, true, false>), grid, blk, 0, s, h->geo, nblk, in, wl, out_act, out_f, mask,
                       scal, i_s, rin, skip, scal2, i_s2);
  else
    hipLaunchKernelGGL((k_conv_ws<NW, EPI_MASK, false, false>), grid, blk, 0, s, h->geo, nblk, in, wl, out_act, out_f,
                       mask, scal, i_s, rin, skip, scal2, i_s2);
}

static void conv_launch(qxd_handle* h, int layer, const uint16_t* in, const uint16_t* W, int nout, int epi,
                        uint16_t* out_act, float* out_f, const uint16_t* mask, const double* scal, int i_s,
                        hipStream_t s, const float* rin = nullptr, float skip = 0.f, const double* scal2 = nullptr,
                        int i_s2 = 0, const qxd_nn* net = nullptr) {
  const uint16_t* wl = W + (size_t)layer * NN_LAYER_W;
  if (net && net->blk) {
    conv_launch_blk(h, net, layer, in, wl, epi, out_act, out_f, mask, scal, i_s, s, rin, skip, scal2, i_s2);
    return;
  }
  int waves = div_up(nout, 64);
  dim3 grid(div_up(waves, 4));
  if (epi == EPI_RELU) {
    if (layer == 0)
      hipLaunchKernelGGL((k_conv<EPI_RELU, true>), grid, dim3(256), 0, s, h->geo, in, wl, nout, out_act, out_f, mask,
                         scal, i_s, rin, skip, scal2, i_s2);
    else
      hipLaunchKernelGGL((k_conv<EPI_RELU, false>), grid, dim3(256), 0, s, h->geo, in, wl, nout, out_act, out_f, mask,
                         scal, i_s, rin, skip, scal2, i_s2);
  } else if (epi == EPI_SPINOR) {
    hipLaunchKernelGGL((k_conv<EPI_SPINOR, false>), grid, dim3(256), 0, s, h->geo, in, wl, nout, out_act, out_f, mask,
                       scal, i_s, rin, skip, scal2, i_s2);
  } else {
    hipLaunchKernelGGL((k_conv<EPI_MASK, false>), grid, dim3(256), 0, s, h->geo, in, wl, nout, out_act, out_f, mask,
                       scal, i_s, rin, skip, scal2, i_s2);
  }
}

// The tiled convolution runs when the 4 x 4 x 4 x 8 blocks divide the extended
// lattice; otherwise the per-site gather kernel does.
static bool nn_blocks_fit(const Geo& g) {
  return g.Le0 % NnBlock::B0 == 0 && g.Le1 % NnBlock::B1 == 0 && g.Le2 % NnBlock::B2 == 0 && g.Le3 % NnBlock::B3 == 0;
}

// free the buffers at ptrs and null them (a partly failed allocation leaves
// nothing behind, so that the next call allocates again)
static void nn_free_all(std::initializer_list<void**> ptrs) {
  for (void** p : ptrs) {
    if (*p) (void)hipFree(*p);
    *p = nullptr;
  }
}

static qxd_status nn_alloc_act(qxd_nn* net, hipStream_t s) {
  if (net->a0) return QXD_OK;
  size_t bytes = (size_t)net->h->V * NN_C * sizeof(uint16_t);
  if (!dev_alloc(&net->a0, bytes) || !dev_alloc(&net->a1, bytes) || !dev_alloc(&net->a2, bytes)) {
    nn_free_all({(void**)&net->a0, (void**)&net->a1, (void**)&net->a2});
    return QXD_ENOMEM;
  }
  // the odd sites and channels 24..31 of a0 are never written: zero once
  QXD_HIP(hipMemsetAsync(net->a0, 0, bytes, s));
  return QXD_OK;
}

static qxd_status nn_alloc_train(qxd_nn* net, hipStream_t s) {
  QXD_TRY(nn_alloc_act(net, s));
  if (net->g3) return QXD_OK;
  qxd_handle* h = net->h;
  size_t bytes = (size_t)h->V * NN_C * sizeof(uint16_t);
  net->nchunk = div_up(h->V, kWgChunk);
  if (!dev_alloc(&net->g3, bytes) || !dev_alloc(&net->gA, bytes) || !dev_alloc(&net->gB, bytes) ||
      !dev_alloc(&net->y, (size_t)h->Ve * 24 * sizeof(float)) ||
      !dev_alloc(&net->dv, (size_t)h->Ve * 24 * sizeof(float)) ||
      !dev_alloc(&net->dz, (size_t)h->Ve * 24 * sizeof(float)) ||
      !dev_alloc(&net->part, (size_t)net->nchunk * NN_TAPS * NN_C * NN_C * sizeof(float))) {
    nn_free_all({(void**)&net->g3, (void**)&net->gA, (void**)&net->gB, (void**)&net->y, (void**)&net->dv,
                 (void**)&net->dz, (void**)&net->part});
    return QXD_ENOMEM;
  }
  // the odd half of g3 is never written: zero once
  QXD_HIP(hipMemsetAsync(net->g3, 0, bytes, s));
  return QXD_OK;
}

// forward pass on r (F32 even half): activations a0, a1, a2 and output
// out = scale * N(r / |r|) (scale = |r| when with_norm, else 1 and no input scaling)
static qxd_status nn_forward(qxd_handle* h, qxd_nn* net, const float4* r, float* out, bool with_norm, hipStream_t s) {
  QXD_TRY(nn_alloc_act(net, s));
  if (with_norm) blas_norm2<float4>(h, r, (size_t)6 * h->Ve, h->scal + S_NN, s);
  hipLaunchKernelGGL(k_nn_embed, dim3(div_up(h->Ve, 256)), dim3(256), 0, s, h->geo, r,
                     with_norm ? h->scal : nullptr, S_NN, net->a0);
  conv_launch(h, 0, net->a0, net->wf, (int)h->V, EPI_RELU, net->a1, nullptr, nullptr, nullptr, 0, s, nullptr, 0.f,
              nullptr, 0, net);
  conv_launch(h, 1, net->a1, net->wf, (int)h->V, EPI_RELU, net->a2, nullptr, nullptr, nullptr, 0, s, nullptr, 0.f,
              nullptr, 0, net);
  conv_launch(h, 2, net->a2, net->wf, (int)h->Ve, EPI_SPINOR, nullptr, out, nullptr, with_norm ? h->scal : nullptr,
              S_NN, s, net->skip != 0.f ? reinterpret_cast<const float*>(r) : nullptr, net->skip,
              with_norm ? nullptr : h->scal, S_NN, net);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

qxd_status nn_apply_internal(qxd_handle* h, qxd_nn* net, float4* out_e, const float4* in_e, hipStream_t s) {
  if (!net || net->h != h) return QXD_EINVAL;
  return nn_forward(h, net, in_e, reinterpret_cast<float*>(out_e), true, s);
}

// loss of one pair (r, e) and, with `backward`, accumulation of its weight
// gradient (scaled by invB) into net->grad.  Device scalars: slot + 0 = |r|^2,
// slot + 1 = |e|^2, slot + 2 = |N(rhat) - ehat|^2 |e|^2 / |r|^2... stored raw as
// |N(rhat) - e/|r||^2; the pair loss is scal[slot+2] scal[slot] / scal[slot+1].
static qxd_status nn_pair(qxd_handle* h, qxd_nn* net, const float4* r, const float4* e, double invB, int slot,
                          int kind, bool backward, hipStream_t s) {
  size_t nw = (size_t)6 * h->Ve;
  blas_norm2<float4>(h, r, nw, h->scal + slot, s);
  blas_norm2<float4>(h, e, nw, h->scal + slot + 1, s);
  // forward on r / |r| (scale 1 at the output): y = N(rhat)
  hipLaunchKernelGGL(k_nn_embed, dim3(div_up(h->Ve, 256)), dim3(256), 0, s, h->geo, r, h->scal, slot, net->a0);
  conv_launch(h, 0, net->a0, net->wf, (int)h->V, EPI_RELU, net->a1, nullptr, nullptr, nullptr, 0, s, nullptr, 0.f,
              nullptr, 0, net);
  conv_launch(h, 1, net->a1, net->wf, (int)h->V, EPI_RELU, net->a2, nullptr, nullptr, nullptr, 0, s, nullptr, 0.f,
              nullptr, 0, net);
  conv_launch(h, 2, net->a2, net->wf, (int)h->Ve, EPI_SPINOR, nullptr, net->y, nullptr, nullptr, 0, s,
              net->skip != 0.f ? reinterpret_cast<const float*>(r) : nullptr, net->skip, h->scal, slot, net);
  // output gradient and loss partials
  int G = div_up(h->Ve, 256);
  if (kind == 0) {
    hipLaunchKernelGGL(k_nn_lossgrad, dim3(G), dim3(256), 0, s, h->geo, (const float4*)net->y, e, h->scal, slot,
                       slot + 1, invB, net->g3, h->partial);
    launch_final_sum(h->partial, G, 1, G, h->scal + slot + 2, s);
  } else {
    // u = y - ehat;  v = D_hat u (|v|^2 -> slot + 2);  g = (2/B) D_hat^+ v
    hipLaunchKernelGGL(k_nn_err, dim3(div_up(6 * h->Ve, 256)), dim3(256), 0, s, (int)h->Ve, (float4*)net->y, e,
                       h->scal, slot);
    QXD_TRY(qxd_schur_apply(h, QXD_F32, 0, net->dv, net->y, h->scal + slot + 2, s));
    if (backward) {
      QXD_TRY(qxd_schur_apply(h, QXD_F32, 1, net->dz, net->dv, nullptr, s));
      hipLaunchKernelGGL(k_nn_embed_grad, dim3(G), dim3(256), 0, s, (int)h->Ve, (const float4*)net->dz,
                         (float)(2.0 * invB), net->g3);
    }
  }
  if (!backward) return QXD_OK;
  // layer 3: weight gradient over the even sites, data gradient masked by a2 > 0
  dim3 wg(net->nchunk, div_up(NN_TAPS, 4));
  dim3 wg_e(div_up(h->Ve, kWgChunk), div_up(NN_TAPS, 4));
  hipLaunchKernelGGL(k_conv_wgrad, wg_e, dim3(256), 0, s, h->geo, net->g3, net->a2, (int)h->Ve, kWgChunk, net->part);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(div_up(NN_TAPS * 24 * 32, 256)), dim3(256), 0, s, net->part,
                     (int)wg_e.x, 32, 24, kOff[2], net->grad);
  conv_launch(h, 2, net->g3, net->wa, (int)h->V, EPI_MASK, net->gA, nullptr, net->a2, nullptr, 0, s, nullptr, 0.f,
              nullptr, 0, net);
  // layer 2
  hipLaunchKernelGGL(k_conv_wgrad, wg, dim3(256), 0, s, h->geo, net->gA, net->a1, (int)h->V, kWgChunk, net->part);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(div_up(NN_TAPS * 32 * 32, 256)), dim3(256), 0, s, net->part, net->nchunk,
                     32, 32, kOff[1], net->grad);
  conv_launch(h, 1, net->gA, net->wa, (int)h->V, EPI_MASK, net->gB, nullptr, net->a1, nullptr, 0, s, nullptr, 0.f,
              nullptr, 0, net);
  // layer 1
  hipLaunchKernelGGL(k_conv_wgrad, wg, dim3(256), 0, s, h->geo, net->gB, net->a0, (int)h->V, kWgChunk, net->part);
  hipLaunchKernelGGL(k_wgrad_reduce, dim3(div_up(NN_TAPS * 32 * 24, 256)), dim3(256), 0, s, net->part, net->nchunk,
                     24, 32, kOff[0], net->grad);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

static double pair_loss(const qxd_handle* h, int slot, int kind) {
  if (kind == 0) return h->scal_host[slot + 2] * h->scal_host[slot] / h->scal_host[slot + 1];
  return h->scal_host[slot + 2];
}

extern "C" qxd_status qxd_nn_create(qxd_handle* h, qxd_nn** out) {
  if (!h || !out) return QXD_EINVAL;
  qxd_nn* net = new (std::nothrow) qxd_nn();
  if (!net) return QXD_ENOMEM;
  net->h = h;
  const char* gather = getenv("QXD_NN_GATHER");
  net->blk = !(gather && gather[0] == '1') && nn_blocks_fit(h->geo);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&net->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || net->ncu < 1)
    net->ncu = 1;
  size_t n = QXD_NN_NWEIGHTS;
  if (!dev_alloc(&net->w, n * 4) || !dev_alloc(&net->m, n * 4) ||
      !dev_alloc(&net->v, n * 4) || !dev_alloc(&net->grad, n * 4) ||
      !dev_alloc(&net->wf, (size_t)3 * NN_LAYER_W * 2) ||
      !dev_alloc(&net->wa, (size_t)3 * NN_LAYER_W * 2)) {
    qxd_nn_destroy(net);
    return QXD_ENOMEM;
  }
  if (hipMemset(net->w, 0, n * 4) != hipSuccess || hipMemset(net->m, 0, n * 4) != hipSuccess ||
      hipMemset(net->v, 0, n * 4) != hipSuccess || hipMemset(net->grad, 0, n * 4) != hipSuccess) {
    qxd_nn_destroy(net);
    return QXD_EHIP;
  }
  if (nn_repack(net, nullptr) != QXD_OK || hipDeviceSynchronize() != hipSuccess) {
    qxd_nn_destroy(net);
    return QXD_EHIP;
  }
  *out = net;
  return QXD_OK;
}

extern "C" qxd_status qxd_nn_destroy(qxd_nn* net) {
  if (!net) return QXD_EINVAL;
  (void)hipDeviceSynchronize();
  void* ptrs[] = {net->w, net->wf, net->wa, net->m, net->v, net->grad, net->a0, net->a1,
                  net->a2, net->g3, net->gA, net->gB, net->y, net->part, net->dv, net->dz};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  delete net;
  return QXD_OK;
}

extern "C" qxd_status qxd_nn_set_skip(qxd_nn* net, double skip) {
  if (!net || !std::isfinite(skip)) return QXD_EINVAL;
  net->skip = (float)skip;
  return QXD_OK;
}

extern "C" qxd_status qxd_nn_set_weights(qxd_nn* net, const float* w) {
  if (!net || !w) return QXD_EINVAL;
  // non-finite weights are accepted: the solver detects and drops the
  // directions such a network produces
  QXD_HIP(hipMemcpy(net->w, w, QXD_NN_NWEIGHTS * sizeof(float), hipMemcpyHostToDevice));
  QXD_HIP(hipMemset(net->m, 0, QXD_NN_NWEIGHTS * 4));
  QXD_HIP(hipMemset(net->v, 0, QXD_NN_NWEIGHTS * 4));
  net->t = 0;
  QXD_TRY(nn_repack(net, nullptr));
  QXD_HIP(hipDeviceSynchronize());
  return QXD_OK;
}

extern "C" qxd_status qxd_nn_get_weights(qxd_nn* net, float* w) {
  if (!net || !w) return QXD_EINVAL;
  QXD_HIP(hipDeviceSynchronize());
  QXD_HIP(hipMemcpy(w, net->w, QXD_NN_NWEIGHTS * sizeof(float), hipMemcpyDeviceToHost));
  return QXD_OK;
}

// Network file: 8-byte tag "QXDNNW01", int32 weight count, float32 skip,
// uint32 FNV-1a hash of the weight bytes, uint32 zero, then the FP32 master
// weights in the packed order of the header (host byte order, little-endian
// on every machine this library runs on).
static const char kNnTag[8] = {'Q', 'X', 'D', 'N', 'N', 'W', '0', '1'};

static uint32_t fnv1a(const unsigned char* p, size_t n) {
  uint32_t x = 2166136261u;
  for (size_t i = 0; i < n; ++i) x = (x ^ p[i]) * 16777619u;
  return x;
}

extern "C" qxd_status qxd_nn_save(qxd_nn* net, const char* path) {
  if (!net || !path) return QXD_EINVAL;
  std::vector<float> w(QXD_NN_NWEIGHTS);
  QXD_HIP(hipDeviceSynchronize());
  QXD_HIP(hipMemcpy(w.data(), net->w, QXD_NN_NWEIGHTS * sizeof(float), hipMemcpyDeviceToHost));
  const size_t nb = w.size() * sizeof(float);
  int32_t count = QXD_NN_NWEIGHTS;
  uint32_t hash = fnv1a(reinterpret_cast<const unsigned char*>(w.data()), nb), zero = 0;
  FILE* f = std::fopen(path, "wb");
  if (!f) return QXD_EIO;
  bool ok = std::fwrite(kNnTag, 1, 8, f) == 8 && std::fwrite(&count, 4, 1, f) == 1 &&
            std::fwrite(&net->skip, 4, 1, f) == 1 && std::fwrite(&hash, 4, 1, f) == 1 &&
            std::fwrite(&zero, 4, 1, f) == 1 && std::fwrite(w.data(), 1, nb, f) == nb;
  ok = (std::fclose(f) == 0) && ok;
  return ok ? QXD_OK : QXD_EIO;
}

extern "C" qxd_status qxd_nn_load(qxd_nn* net, const char* path) {
  if (!net || !path) return QXD_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return QXD_EIO;
  char tag[8];
  int32_t count = 0;
  float skip = 0.f;
  uint32_t hash = 0, zero = 1;
  std::vector<float> w(QXD_NN_NWEIGHTS);
  const size_t nb = w.size() * sizeof(float);
  bool ok = std::fread(tag, 1, 8, f) == 8 && std::memcmp(tag, kNnTag, 8) == 0 && std::fread(&count, 4, 1, f) == 1 &&
            count == QXD_NN_NWEIGHTS && std::fread(&skip, 4, 1, f) == 1 && std::fread(&hash, 4, 1, f) == 1 &&
            std::fread(&zero, 4, 1, f) == 1 && zero == 0 && std::fread(w.data(), 1, nb, f) == nb &&
            std::fgetc(f) == EOF;
  std::fclose(f);
  if (!ok || fnv1a(reinterpret_cast<const unsigned char*>(w.data()), nb) != hash || !std::isfinite(skip))
    return QXD_EIO;
  QXD_TRY(qxd_nn_set_weights(net, w.data()));
  net->skip = skip;
  return QXD_OK;
}

extern "C" qxd_status qxd_nn_apply(qxd_handle* h, qxd_nn* net, void* out_e, const void* in_e, void* stream) {
  if (!h || !net || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  return nn_apply_internal(h, net, (float4*)out_e, (const float4*)in_e, as_stream(stream));
}

extern "C" qxd_status qxd_nn_loss_grad(qxd_handle* h, qxd_nn* net, const void* r, const void* e, int n,
                                       int loss_kind, double* loss, float* grad, void* stream) {
  if (!h || !net || !r || !e || n < 1 || net->h != h || loss_kind < 0 || loss_kind > 1) return QXD_EINVAL;
  if (loss_kind == 1 && !h->has_inverse) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  QXD_TRY(nn_alloc_train(net, s));
  QXD_HIP(hipMemsetAsync(net->grad, 0, QXD_NN_NWEIGHTS * 4, s));
  size_t half = (size_t)6 * h->Ve;
  double total = 0.0;
  for (int i = 0; i < n; ++i) {
    QXD_TRY(nn_pair(h, net, (const float4*)r + i * half, (const float4*)e + i * half, 1.0 / n, S_NN, loss_kind, true,
                    s));
    QXD_HIP(hipMemcpyAsync(h->scal_host + S_NN, h->scal + S_NN, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    QXD_HIP(hipStreamSynchronize(s));
    total += pair_loss(h, S_NN, loss_kind) / n;
  }
  if (loss) *loss = total;
  if (grad) {
    QXD_HIP(hipMemcpyAsync(grad, net->grad, QXD_NN_NWEIGHTS * 4, hipMemcpyDeviceToHost, s));
    QXD_HIP(hipStreamSynchronize(s));
  }
  return QXD_OK;
}

static uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Adam on minibatches of pairs; the last p->holdout pairs are only evaluated.
extern "C" qxd_status qxd_nn_train(qxd_handle* h, qxd_nn* net, const qxd_train_params* p, const void* r, const void* e,
                                   int npairs, qxd_train_stats* stats, void* stream) {
  auto t0 = std::chrono::steady_clock::now();
  if (!h || !net || !p || !r || !e || net->h != h) return QXD_EINVAL;
  int ntrain = npairs - std::max(0, p->holdout);
  if (ntrain < 1 || p->batch < 1 || p->batch > 64 || p->epochs < 1 || p->loss < 0 || p->loss > 1) return QXD_EINVAL;
  if (p->loss == 1 && !h->has_inverse) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  QXD_TRY(nn_alloc_train(net, s));
  size_t half = (size_t)6 * h->Ve;
  const float4* R = (const float4*)r;
  const float4* E = (const float4*)e;
  std::vector<int> order(ntrain);
  for (int i = 0; i < ntrain; ++i) order[i] = i;
  uint64_t seed = p->seed;
  qxd_train_stats st{};
  const int base = S_NN + 8;
  for (int ep = 0; ep < p->epochs; ++ep) {
    for (int i = ntrain - 1; i > 0; --i) std::swap(order[i], order[(int)(splitmix64(seed) % (uint64_t)(i + 1))]);
    double ep_loss = 0.0;
    for (int b0 = 0; b0 < ntrain; b0 += p->batch) {
      int nb = std::min(p->batch, ntrain - b0);
      QXD_HIP(hipMemsetAsync(net->grad, 0, QXD_NN_NWEIGHTS * 4, s));
      for (int k = 0; k < nb; ++k) {
        int idx = order[b0 + k];
        QXD_TRY(nn_pair(h, net, R + idx * half, E + idx * half, 1.0 / nb, base + 3 * k, p->loss, true, s));
      }
      net->t++;
      float c1 = 1.f - (float)std::pow(p->beta1, (double)net->t), c2 = 1.f - (float)std::pow(p->beta2, (double)net->t);
      hipLaunchKernelGGL(k_adam, dim3(div_up(QXD_NN_NWEIGHTS, 256)), dim3(256), 0, s, net->w, net->grad, net->m,
                         net->v, (int)QXD_NN_NWEIGHTS, (float)p->lr, (float)p->beta1, (float)p->beta2, (float)p->eps,
                         c1, c2);
      QXD_TRY(nn_repack(net, s));
      QXD_HIP(hipMemcpyAsync(h->scal_host + base, h->scal + base, 3 * nb * sizeof(double), hipMemcpyDeviceToHost, s));
      QXD_HIP(hipStreamSynchronize(s));
      for (int k = 0; k < nb; ++k) ep_loss += pair_loss(h, base + 3 * k, p->loss);
      st.steps++;
    }
    ep_loss /= ntrain;
    if (!std::isfinite(ep_loss)) return QXD_ENAN;
    if (ep == 0) st.loss_first = ep_loss;
    st.loss_last = ep_loss;
  }
  double hl = 0.0;
  int nh = npairs - ntrain;
  for (int i = 0; i < nh; ++i) {
    QXD_TRY(nn_pair(h, net, R + (ntrain + i) * half, E + (ntrain + i) * half, 1.0, base, p->loss, false, s));
    QXD_HIP(hipMemcpyAsync(h->scal_host + base, h->scal + base, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    QXD_HIP(hipStreamSynchronize(s));
    hl += pair_loss(h, base, p->loss) / nh;
  }
  st.holdout_loss = nh > 0 ? hl : 0.0;
  st.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = st;
  return QXD_OK;
}
