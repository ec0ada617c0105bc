// Internal declarations of libqxd (MI355X / gfx950).
//
// Device layouts (Ve = half volume, h = half index of a site within its parity):
//   spinor half field  F64  double2 [12][Ve]      component c = 3 spin + colour
//                      F32  float4  [6][Ve]       components (2j, 2j+1)
//                      BF16 uint4   [3][Ve]       components 4j..4j+3, bf16 (re, im)
//   links V = U z^qhat  [parity][mu][9][Ve] of double2; float2 and bf16x2 (uint32) regrouped per
//                       (parity, mu) into 16-byte words of 2 or 4 entries per site (see lk_load),
//                       row-major colour matrix, entry k = 3 row + col
//   clover blocks       [36][Ve] double2 or [18][Ve] float4 per parity: two
//                       Hermitian 6x6 blocks (upper, lower chirality), each 36
//                       reals: 6 real diagonal entries, then the 15 upper
//                       off-diagonal complex entries (0,1),(0,2),..,(4,5).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "qxd.h"

#define QXD_BLOCK 256

// ---------------------------------------------------------------------------
// complex arithmetic

template <class T>
struct cx {
  T re, im;
};

template <class T>
__host__ __device__ inline cx<T> mk(T r, T i) { return cx<T>{r, i}; }
template <class T>
__host__ __device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return {a.re + b.re, a.im + b.im}; }
template <class T>
__host__ __device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return {a.re - b.re, a.im - b.im}; }
template <class T>
__host__ __device__ inline cx<T> operator-(cx<T> a) { return {-a.re, -a.im}; }
template <class T>
__host__ __device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <class T>
__host__ __device__ inline cx<T> operator*(T s, cx<T> a) { return {s * a.re, s * a.im}; }
template <class T>
__host__ __device__ inline cx<T> conj(cx<T> a) { return {a.re, -a.im}; }
// i * a
template <class T>
__host__ __device__ inline cx<T> ti(cx<T> a) { return {-a.im, a.re}; }
// conj(a) * b
template <class T>
__host__ __device__ inline cx<T> cmul_conj(cx<T> a, cx<T> b) {
  return {a.re * b.re + a.im * b.im, a.re * b.im - a.im * b.re};
}
template <class T>
__host__ __device__ inline T norm2(cx<T> a) { return a.re * a.re + a.im * a.im; }

// ---------------------------------------------------------------------------
// geometry of the extended lattice (C* orbifold, even-odd half indices)

struct Geo {
  int Le0, Le1, Le2, Le3;  // extended extents (Le1 = 2 L1 with C*)
  int L1;                  // physical L1: the shift of a C* boundary crossing in k = 2, 3
  int cstar;               // 0..3
  int tanti;               // fermion sign -1 on the time wrap
  int L3h;                 // Le3 / 2
  int Ve;                  // half volume
  int tchunk;              // workgroup -> lattice tile order (see site_tile)
  int tile0, ntile;        // Schur passes: launch covers tiles tile0 + [0, grid) mod ntile (ntile 0: tile0 = 0)
  int plain_st;            // Schur passes store t_o and chi plainly (1) or with the non-temporal hint (0, default)
};

// Coordinates of the site with half index h in parity p.
__device__ inline void geo_decode(const Geo& g, int p, int h, int& x0, int& x1, int& x2, int& x3) {
  int x3h = h % g.L3h;
  int q = h / g.L3h;
  x2 = q % g.Le2;
  q /= g.Le2;
  x1 = q % g.Le1;
  x0 = q / g.Le1;
  x3 = 2 * x3h + ((p + x0 + x1 + x2) & 1);
}

__device__ inline int geo_half(const Geo& g, int x0, int x1, int x2, int x3) {
  return (x3 >> 1) + g.L3h * (x2 + g.Le2 * (x1 + g.Le1 * x0));
}

// x1 moved by L1 on the doubled direction (period 2 L1)
__device__ inline int geo_mirror_x1(const Geo& g, int x1) { return x1 >= g.L1 ? x1 - g.L1 : x1 + g.L1; }

// Move x to its neighbour x + DIR e_MU (with C*, crossing the boundary of a
// direction k <= cstar, k >= 2, shifts x1 by L1); *neg set when the hop crosses
// the antiperiodic time boundary.
template <int MU, int DIR>
__device__ inline void geo_step(const Geo& g, int& x0, int& x1, int& x2, int& x3, bool& neg) {
  neg = false;
  if (MU == 0) {
    x0 += DIR;
    if (x0 < 0) { x0 += g.Le0; neg = g.tanti; }
    else if (x0 >= g.Le0) { x0 -= g.Le0; neg = g.tanti; }
  } else if (MU == 1) {
    x1 += DIR;
    if (x1 < 0) x1 += g.Le1;
    else if (x1 >= g.Le1) x1 -= g.Le1;
  } else if (MU == 2) {
    x2 += DIR;
    if (x2 < 0 || x2 >= g.Le2) {
      x2 = x2 < 0 ? x2 + g.Le2 : x2 - g.Le2;
      if (g.cstar >= 2) x1 = geo_mirror_x1(g, x1);
    }
  } else {
    x3 += DIR;
    if (x3 < 0 || x3 >= g.Le3) {
      x3 = x3 < 0 ? x3 + g.Le3 : x3 - g.Le3;
      if (g.cstar >= 3) x1 = geo_mirror_x1(g, x1);
    }
  }
}

// Half index of the neighbour x + DIR e_MU
template <int MU, int DIR>
__device__ inline int geo_nb(const Geo& g, int x0, int x1, int x2, int x3, bool& neg) {
  geo_step<MU, DIR>(g, x0, x1, x2, x3, neg);
  return geo_half(g, x0, x1, x2, x3);
}

// Order in which workgroups walk the lattice.  The hardware hands workgroup b
// to XCD b % 8.  With tchunk = K > 0 the walk proceeds in windows of 8K
// consecutive tiles; inside a window each XCD takes K consecutive tiles, so the
// spatial neighbours of a tile mostly sit in the same XCD's L2, while the whole
// GPU advances through the lattice together and the time-direction neighbours
// (two time slices apart) are still in the last-level cache when read again.
// tchunk = 0: plain order; tchunk < 0: each XCD owns one contiguous eighth.
__device__ inline int site_tile(int b, int G, int K) {
  if (K == 0) return b;
  if (K < 0) {
    int per = G >> 3, rem = G & 7;
    int xcd = b & 7, idx = b >> 3;
    return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
  }
  int win = 8 * K;
  int w = b / win;
  if ((w + 1) * win > G) return b;  // ragged last window: plain order
  int r = b - w * win;
  return w * win + (r & 7) * K + (r >> 3);
}

// ---------------------------------------------------------------------------
// bfloat16 (round to nearest even; NaN kept quiet)

__host__ __device__ inline uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __builtin_bit_cast(uint32_t, f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (u >> 16) | 0x40u;
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__host__ __device__ inline float bf16_bits_to_f32(uint32_t b) { return __builtin_bit_cast(float, b << 16); }
__host__ __device__ inline uint32_t pack_bf16x2(float lo, float hi) {
  return f32_to_bf16_bits(lo) | (f32_to_bf16_bits(hi) << 16);
}
__host__ __device__ inline float bf16lo(uint32_t w) { return __builtin_bit_cast(float, w << 16); }
__host__ __device__ inline float bf16hi(uint32_t w) { return __builtin_bit_cast(float, w & 0xffff0000u); }

// ---------------------------------------------------------------------------
// spinor storage: load / store 12 components of site h

__device__ inline void sp_load(const double2* __restrict__ f, size_t Ve, int h, cx<double> s[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    double2 v = f[c * Ve + h];
    s[c] = mk(v.x, v.y);
  }
}
__device__ inline void sp_store(double2* __restrict__ f, size_t Ve, int h, const cx<double> s[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) f[c * Ve + h] = make_double2(s[c].re, s[c].im);
}
// Non-temporal stores, for the outputs of the Schur passes: measured faster than
// plain stores for both passes on gfx950, also for t_o, which the second pass
// reads back.
typedef double nt_st_d2 __attribute__((ext_vector_type(2)));
typedef float nt_st_f4 __attribute__((ext_vector_type(4)));
__device__ inline void sp_store_nt(double2* __restrict__ f, size_t Ve, int h, const cx<double> s[12]) {
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    nt_st_d2 v = {s[c].re, s[c].im};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_st_d2*>(&f[c * Ve + h]));
  }
}
__device__ inline void sp_store_nt(float4* __restrict__ f, size_t Ve, int h, const cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    nt_st_f4 v = {s[2 * j].re, s[2 * j].im, s[2 * j + 1].re, s[2 * j + 1].im};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_st_f4*>(&f[j * Ve + h]));
  }
}
__device__ inline void sp_load(const float4* __restrict__ f, size_t Ve, int h, cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    float4 v = f[j * Ve + h];
    s[2 * j] = mk(v.x, v.y);
    s[2 * j + 1] = mk(v.z, v.w);
  }
}
__device__ inline void sp_store(float4* __restrict__ f, size_t Ve, int h, const cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 6; ++j)
    f[j * Ve + h] = make_float4(s[2 * j].re, s[2 * j].im, s[2 * j + 1].re, s[2 * j + 1].im);
}
__device__ inline void sp_load(const uint4* __restrict__ f, size_t Ve, int h, cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    uint4 v = f[j * Ve + h];
    s[4 * j + 0] = mk(bf16lo(v.x), bf16hi(v.x));
    s[4 * j + 1] = mk(bf16lo(v.y), bf16hi(v.y));
    s[4 * j + 2] = mk(bf16lo(v.z), bf16hi(v.z));
    s[4 * j + 3] = mk(bf16lo(v.w), bf16hi(v.w));
  }
}
__device__ inline void sp_store(uint4* __restrict__ f, size_t Ve, int h, const cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    uint4 v;
    v.x = pack_bf16x2(s[4 * j].re, s[4 * j].im);
    v.y = pack_bf16x2(s[4 * j + 1].re, s[4 * j + 1].im);
    v.z = pack_bf16x2(s[4 * j + 2].re, s[4 * j + 2].im);
    v.w = pack_bf16x2(s[4 * j + 3].re, s[4 * j + 3].im);
    f[j * Ve + h] = v;
  }
}
typedef uint32_t nt_st_u4 __attribute__((ext_vector_type(4)));
__device__ inline void sp_store_nt(uint4* __restrict__ f, size_t Ve, int h, const cx<float> s[12]) {
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    nt_st_u4 v = {pack_bf16x2(s[4 * j].re, s[4 * j].im), pack_bf16x2(s[4 * j + 1].re, s[4 * j + 1].im),
                  pack_bf16x2(s[4 * j + 2].re, s[4 * j + 2].im), pack_bf16x2(s[4 * j + 3].re, s[4 * j + 3].im)};
    __builtin_nontemporal_store(v, reinterpret_cast<nt_st_u4*>(&f[j * Ve + h]));
  }
}

// link storage: 9 entries of the colour matrix of link (parity array, mu, h)
// Links and clover blocks are read once per pass: load them with the
// non-temporal hint so that they do not evict the neighbour spinors, which are
// read by up to eight sites, from the L2.
typedef double nt_d2 __attribute__((ext_vector_type(2)));
typedef float nt_f2 __attribute__((ext_vector_type(2)));
typedef float nt_f4 __attribute__((ext_vector_type(4)));
__device__ inline double2 ld_stream(const double2* p) {
  nt_d2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(p));
  return make_double2(v.x, v.y);
}
__device__ inline float2 ld_stream(const float2* p) {
  nt_f2 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f2*>(p));
  return make_float2(v.x, v.y);
}
__device__ inline float4 ld_stream(const float4* p) {
  nt_f4 v = __builtin_nontemporal_load(reinterpret_cast<const nt_f4*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}
__device__ inline uint32_t ld_stream(const uint32_t* p) { return __builtin_nontemporal_load(p); }
__device__ inline void st_stream(double2* p, double2 a) {
  nt_d2 v = {a.x, a.y};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_d2*>(p));
}
__device__ inline void st_stream(float4* p, float4 a) {
  nt_f4 v = {a.x, a.y, a.z, a.w};
  __builtin_nontemporal_store(v, reinterpret_cast<nt_f4*>(p));
}

__device__ inline void lk_load(const double2* __restrict__ V, size_t Ve, int mu, int h, cx<double> u[9]) {
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 v = ld_stream(&V[(mu * 9 + k) * Ve + h]);
    u[k] = mk(v.x, v.y);
  }
}
// FP32 links: the 9 Ve float2 of (parity, mu) hold entries 2j, 2j + 1 of every
// link as one 16-byte word per h in the j-th quarter of the first 8 Ve
// (j < 4), then entry 8 as an 8-byte word per h: one link in five loads
__device__ inline size_t lk32_index(size_t Ve, int k, size_t h) {
  return k < 8 ? (size_t)(k >> 1) * 2 * Ve + 2 * h + (k & 1) : 8 * Ve + h;
}
__device__ inline void lk_load(const float2* __restrict__ V, size_t Ve, int mu, int h, cx<float> u[9]) {
  const float2* base = V + (size_t)mu * 9 * Ve;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    float4 v = ld_stream(reinterpret_cast<const float4*>(base + (size_t)j * 2 * Ve) + h);
    u[2 * j] = mk(v.x, v.y);
    u[2 * j + 1] = mk(v.z, v.w);
  }
  float2 v = ld_stream(base + 8 * Ve + h);
  u[8] = mk(v.x, v.y);
}
// bf16 links: the 9 Ve words of (parity, mu) hold entries 0..3 of every link
// as one 16-byte word per h, then entries 4..7 likewise, then entry 8 as a
// 4-byte word per h: one link in three loads instead of nine
typedef uint32_t nt_u4 __attribute__((ext_vector_type(4)));
__device__ inline void lk_load(const uint32_t* __restrict__ V, size_t Ve, int mu, int h, cx<float> u[9]) {
  const uint32_t* base = V + (size_t)mu * 9 * Ve;
  const nt_u4 a = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(base) + h);
  const nt_u4 b = __builtin_nontemporal_load(reinterpret_cast<const nt_u4*>(base + 4 * Ve) + h);
  const uint32_t c = ld_stream(base + 8 * Ve + h);
  u[0] = mk(bf16lo(a.x), bf16hi(a.x));
  u[1] = mk(bf16lo(a.y), bf16hi(a.y));
  u[2] = mk(bf16lo(a.z), bf16hi(a.z));
  u[3] = mk(bf16lo(a.w), bf16hi(a.w));
  u[4] = mk(bf16lo(b.x), bf16hi(b.x));
  u[5] = mk(bf16lo(b.y), bf16hi(b.y));
  u[6] = mk(bf16lo(b.z), bf16hi(b.z));
  u[7] = mk(bf16lo(b.w), bf16hi(b.w));
  u[8] = mk(bf16lo(c), bf16hi(c));
}

// clover storage: two packed Hermitian 6x6 blocks (72 reals)
__device__ inline void cl_load(const double2* __restrict__ C, size_t Ve, int h, double r[72]) {
#pragma unroll
  for (int k = 0; k < 36; ++k) {
    double2 v = ld_stream(&C[k * Ve + h]);
    r[2 * k] = v.x;
    r[2 * k + 1] = v.y;
  }
}
__device__ inline void cl_load(const float4* __restrict__ C, size_t Ve, int h, float r[72]) {
#pragma unroll
  for (int k = 0; k < 18; ++k) {
    float4 v = ld_stream(&C[k * Ve + h]);
    r[4 * k] = v.x;
    r[4 * k + 1] = v.y;
    r[4 * k + 2] = v.z;
    r[4 * k + 3] = v.w;
  }
}

// out[0..5] = H in[0..5] for one packed Hermitian block b (36 reals)
template <class T>
__device__ inline void herm6_mul(const T* b, const cx<T>* in, cx<T>* out) {
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = b[i] * in[i];
  int k = 6;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      cx<T> hij = mk(b[k], b[k + 1]);
      k += 2;
      out[i] = out[i] + hij * in[j];
      out[j] = out[j] + cmul_conj(hij, in[i]);
    }
  }
}

// index of the packed entry (i, j), i < j, within a block
__host__ __device__ constexpr int herm6_off(int i, int j) {
  // entries before row i: sum_{r<i} (5 - r)
  return 6 + 2 * (i * 5 - i * (i - 1) / 2 + (j - i - 1));
}

// ---------------------------------------------------------------------------
// the handle

struct qxd_handle {
  int device = 0;
  qxd_geom g{};
  Geo geo{};
  int64_t V = 0, Ve = 0, Vphys = 0;
  // gauge field on the physical lattice (canonical layout)
  double* Uphys = nullptr;  // [4][Vphys][9] complex
  double* Aphys = nullptr;  // [4][Vphys]
  bool has_gauge = false, has_flavour = false, has_clover = false, has_inverse = false;
  qxd_flavour fl{};
  // combined links V = U z^qhat, [2][4][9][Ve]
  double2* V64 = nullptr;
  float2* V32 = nullptr;
  uint32_t* V16 = nullptr;
  // clover blocks: H on even and odd sites, H^-1 on odd sites
  double2 *He64 = nullptr, *Ho64 = nullptr, *Hi64 = nullptr;
  float4 *He32 = nullptr, *Ho32 = nullptr, *Hi32 = nullptr;
  // odd half-field workspaces for the Schur passes
  double2* t64 = nullptr;
  float4* t32 = nullptr;
  uint4* t16 = nullptr;
  // reductions
  double* partial = nullptr;  // [QXD_MAX_PARTIAL]
  double* scal = nullptr;     // [QXD_NSCAL] device scalars
  double* scal_host = nullptr;  // pinned mirror
  size_t npartial = 0;        // doubles in `partial`
  bool tchunk_env = false;    // walk chunk fixed by QXD_TILE_CHUNK
  int slices_env = -1;        // time slices per Schur chunk fixed by QXD_SCHUR_SLICES (-1: by size)
  unsigned copies = 0;        // CP_* bits: lower-precision operator copies that are current
  uint64_t setup_gen = 0;     // bumped whenever the links or clover blocks are rebuilt
  uint64_t sap_gen = 0;       // SAP's block-order copies: 2 setup_gen + slot order (0: none)
  // solver workspaces (grow-only), indexed by role
  void* ws[64] = {};
  size_t ws_bytes[64] = {};
};

#define QXD_NSCAL 4096
#define QXD_MAX_PARTIAL (64 * 2048)

// device scalar slots
enum {
  S_ZZ0 = 0, S_ZZ1 = 1, S_WW = 2, S_RR = 3, S_NB = 4, S_RT = 5, S_BH = 6, S_ONE = 7,
  S_FRR = 16,            // FGCR |r|^2
  S_FB = 32,             // FGCR |chi_k|^2, k < 64
  S_FC = 128,            // FGCR c_k (complex), k < 64
  S_FR = 1024,           // FGCR R[k][j] (complex), column k at S_FR + 2 k QXD_MAXKV_R
  S_FAL = 3200,          // FGCR solution coefficients (complex)
  S_NN = 3400            // network preconditioner scratch scalars
};
#define QXD_MAXKV_R 32

// hipMalloc that leaves no error behind when it fails: the caller reports
// QXD_ENOMEM, and the launch checks of later calls must not see the failed
// allocation again as a HIP error.
template <class T>
inline bool dev_alloc(T** p, size_t bytes) {
  if (hipMalloc(reinterpret_cast<void**>(p), bytes) == hipSuccess) return true;
  *p = nullptr;
  (void)hipGetLastError();
  return false;
}

// grow-only device workspace number i of at least `bytes`
inline void* ws_get(qxd_handle* h, int i, size_t bytes) {
  if (h->ws_bytes[i] >= bytes) return h->ws[i];
  if (h->ws[i]) (void)hipFree(h->ws[i]);
  h->ws[i] = nullptr;
  h->ws_bytes[i] = 0;
  if (!dev_alloc(&h->ws[i], bytes)) return nullptr;
  h->ws_bytes[i] = bytes;
  return h->ws[i];
}

struct qxd_nn;
struct qxd_dfl;

// error helpers
#define QXD_HIP(call)                            \
  do {                                           \
    hipError_t e_ = (call);                      \
    if (e_ != hipSuccess) return QXD_EHIP;       \
  } while (0)

#define QXD_TRY(call)                            \
  do {                                           \
    qxd_status s_ = (call);                      \
    if (s_ != QXD_OK) return s_;                 \
  } while (0)

inline hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

inline int div_up(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// internal entry points shared between translation units
// out[v] = sum_{i<n} partial[v * stride + i] for v < nvals, summed in a fixed order
void launch_final_sum(const double* partial, int n, int nvals, int stride, double* out, hipStream_t s);
qxd_status qxd_schur_apply(qxd_handle* h, qxd_prec p, int dagger, void* out_e, const void* in_e, double* norm_slot,
                           hipStream_t s);
qxd_status nn_apply_internal(qxd_handle* h, qxd_nn* net, float4* out_e, const float4* in_e, hipStream_t s);
// DFL+SAP preconditioner of the Schur system (dfl.hip): out_e = (M_DFL (in_e, 0))_e
qxd_status dfl_apply_internal(qxd_handle* h, qxd_dfl* d, int nc, int ncy, int nmr, int eo, float4* out_e,
                              const float4* in_e, hipStream_t s);
// SAP (sap.hip) on FP32 fields: out_e = (M_SAP (in_e, in_o))_e, in_o = 0 when
// null, and the odd half of M_SAP (in_e, in_o) into out_o when given
bool sap_supported(const qxd_handle* h);
qxd_status sap_apply_internal(qxd_handle* h, int ncy, int nmr, int eo, float4* out_e, const float4* in_e,
                              hipStream_t s, const float4* in_o = nullptr, float4* out_o = nullptr);
// Lower-precision copies of the operator (links V in FP32 and bf16, clover
// blocks H_e, H_o, H_o^-1 in FP32) are made from the FP64 ones when a call
// first needs them and released by qxd_trim, so that a handle holds only the
// copies the computations it runs use.  ensure_copies makes the `which` copies
// current (QXD_ESTATE if their FP64 source is not set up, QXD_ENOMEM);
// release_copies frees the `which` copies (the caller makes sure no queued
// work still reads them).
enum : unsigned { CP_V32 = 1u, CP_V16 = 2u, CP_HE32 = 4u, CP_HO32 = 8u, CP_HI32 = 16u, CP_ALL = 31u };
qxd_status ensure_copies(qxd_handle* h, unsigned which, hipStream_t s);
void release_copies(qxd_handle* h, unsigned which = CP_ALL);

// device address of the static workspace of qxd_dw_eo_schur_noalloc on
// `device` (the current device), looked up once per device (dirac.hip)
qxd_status scratch_resolve(int device);
qxd_status qxd_schur_apply_mixed(qxd_handle* h, int dagger, float4* out_e, const float4* in_e, double* norm_slot,
                                 hipStream_t s);
