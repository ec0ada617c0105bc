// Wilson-clover operator with SU(3) x U(1)^qhat links on the C* extended lattice
// and its even-odd Schur complement (Sec. 2.3 of arXiv:1908.11673).
//
// Expanding the covariant derivatives of Dw gives, with V = U z^qhat,
//   (D psi)(x) = H(x) psi(x) - (1/2) hop(psi)(x),
//   hop(psi)(x) = sum_mu (1 - g_mu) V(x,mu) psi(x+mu) + (1 + g_mu) V(x-mu,mu)^+ psi(x-mu),
// H = 1/(2 kappa) + SW term (two 6x6 chirality blocks).  Each (1 -+ g_mu) term is
// evaluated on a projected two-spinor: project, multiply by the link, rebuild.
// Hops always connect the two parities, so
//   D_hat psi_e = H_e psi_e - (1/4) hop_eo( H_o^-1 hop_oe(psi_e) ),
// computed in two passes (odd sites, then even sites); D_hat^+ = g5 D_hat g5.
// One work-item per output site; neighbours are found from the site
// coordinates (no neighbour table), including the C* shift of x1 when a hop in
// direction k <= cstar crosses the lattice boundary.
#include <mutex>

#include "wilson_site.hpp"

__device__ inline double block_sum(double v, double* sh) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += sh[i];
  return s;
}

template <class T>
__device__ __forceinline__ double sp_norm2(const cx<T> s[12]) {
  double a = 0.0;
#pragma unroll
  for (int c = 0; c < 12; ++c) a += (double)norm2(s[c]);
  return a;
}

// The outputs of both passes (t_o, chi) are stored either plainly or with the
// non-temporal hint, chosen at run time (Geo::plain_st, QXD_SCHUR_STORES=plain);
// every configuration measured is fastest with the non-temporal stores, also in
// the chunked order where pass 2 reads t_o back soon (FP64 1.70 against
// 1.73 ms).  With the choice in the kernels the compiler schedules the
// bf16-storage passes differently: pass 1 issues its last direction's twelve
// loads together instead of one at a time and needs 146 registers instead of
// 271; bf16 D_hat at 64x64x32x32 went 0.755 -> 0.627 ms (the choice in pass 1)
// -> 0.565 ms (in both passes), the FP64 and FP32 passes unchanged.

// pass 1: t_o = H_o^-1 hop_oe(g5? psi_e)
template <class T, class SPT, class LKT, class CLT, bool DAG>
__global__ __launch_bounds__(QXD_BLOCK) void k_schur1(Geo g, const SPT* __restrict__ in_e, SPT* __restrict__ t_o,
                                                      const LKT* __restrict__ Ve_l, const LKT* __restrict__ Vo_l,
                                                      const CLT* __restrict__ Hi) {
  int tile = site_tile(blockIdx.x, gridDim.x, g.tchunk) + g.tile0;
  if (g.ntile && tile >= g.ntile) tile -= g.ntile;
  int h = tile * QXD_BLOCK + threadIdx.x;
  if (h >= g.Ve) return;
  cx<T> acc[12], out[12];
  hop_site<DAG, T>(g, 1, h, in_e, Vo_l, Ve_l, acc);
  clover_mul<T>(Hi, g.Ve, h, acc, out);
  if (g.plain_st) sp_store(t_o, g.Ve, h, out);
  else sp_store_nt(t_o, g.Ve, h, out);
}

// pass 2: out_e = H_e psi_e - (1/4) g5? hop_eo(t_o); optional block partials of |out|^2
template <class T, class SPT, class LKT, class CLT, bool DAG, bool NORM>
__global__ __launch_bounds__(QXD_BLOCK) void k_schur2(Geo g, const SPT* __restrict__ t_o,
                                                      const SPT* __restrict__ in_e, SPT* __restrict__ out_e,
                                                      const LKT* __restrict__ Ve_l, const LKT* __restrict__ Vo_l,
                                                      const CLT* __restrict__ He, double* __restrict__ partial) {
  __shared__ double sh[QXD_BLOCK / 64];
  int tile = site_tile(blockIdx.x, gridDim.x, g.tchunk) + g.tile0;
  if (g.ntile && tile >= g.ntile) tile -= g.ntile;
  int h = tile * QXD_BLOCK + threadIdx.x;
  double n2 = 0.0;
  if (h < g.Ve) {
    cx<T> acc[12], s[12], c[12];
    hop_site<false, T>(g, 0, h, t_o, Ve_l, Vo_l, acc);
    if (DAG) g5_lower(acc);
    sp_load(in_e, g.Ve, h, s);
    clover_mul<T>(He, g.Ve, h, s, c);
#pragma unroll
    for (int k = 0; k < 12; ++k) c[k] = c[k] - T(0.25) * acc[k];
    if (g.plain_st) sp_store(out_e, g.Ve, h, c);
    else sp_store_nt(out_e, g.Ve, h, c);
    if (NORM) n2 = sp_norm2(c);
  }
  if (NORM) {
    double b = block_sum(n2, sh);
    if (threadIdx.x == 0) partial[tile] = b;
  }
}

// full operator on parity p: out_p = H_p in_p - (1/2) hop(in_q)
template <class T, class SPT, class LKT, class CLT>
__global__ __launch_bounds__(QXD_BLOCK) void k_dw(Geo g, int p, const SPT* __restrict__ in_p,
                                                  const SPT* __restrict__ in_q, SPT* __restrict__ out_p,
                                                  const LKT* __restrict__ Vp, const LKT* __restrict__ Vq,
                                                  const CLT* __restrict__ Hp) {
  int h = site_tile(blockIdx.x, gridDim.x, g.tchunk) * QXD_BLOCK + threadIdx.x;
  if (h >= g.Ve) return;
  cx<T> acc[12], s[12], c[12];
  hop_site<false, T>(g, p, h, in_q, Vp, Vq, acc);
  sp_load(in_p, g.Ve, h, s);
  clover_mul<T>(Hp, g.Ve, h, s, c);
#pragma unroll
  for (int k = 0; k < 12; ++k) c[k] = c[k] - T(0.5) * acc[k];
  sp_store(out_p, g.Ve, h, c);
}

// out_p = C? (base_p + alpha hop(in_q))   (FP64; source preparation and reconstruction)
template <bool CLOV>
__global__ __launch_bounds__(QXD_BLOCK) void k_hop_add(Geo g, int p, const double2* __restrict__ in_q,
                                                       const double2* __restrict__ base, double2* __restrict__ out,
                                                       const double2* __restrict__ Vp, const double2* __restrict__ Vq,
                                                       const double2* __restrict__ C, double alpha) {
  int h = site_tile(blockIdx.x, gridDim.x, g.tchunk) * QXD_BLOCK + threadIdx.x;
  if (h >= g.Ve) return;
  cx<double> acc[12], s[12], c[12];
  hop_site<false, double>(g, p, h, in_q, Vp, Vq, acc);
  sp_load(base, g.Ve, h, s);
#pragma unroll
  for (int k = 0; k < 12; ++k) s[k] = s[k] + alpha * acc[k];
  if (CLOV) {
    clover_mul<double>(C, g.Ve, h, s, c);
    sp_store(out, g.Ve, h, c);
  } else {
    sp_store(out, g.Ve, h, s);
  }
}

// out = C in on one parity
__global__ __launch_bounds__(QXD_BLOCK) void k_clov(int Ve, const double2* __restrict__ in, double2* __restrict__ out,
                                                    const double2* __restrict__ C) {
  int h = blockIdx.x * QXD_BLOCK + threadIdx.x;
  if (h >= Ve) return;
  cx<double> s[12], c[12];
  sp_load(in, Ve, h, s);
  clover_mul<double>(C, Ve, h, s, c);
  sp_store(out, Ve, h, c);
}

// canonical AoS [V][12] complex128 <-> eo SoA of the storage type
template <class SPT, class T>
__global__ __launch_bounds__(QXD_BLOCK) void k_unpack(Geo g, double2* __restrict__ aos, const SPT* __restrict__ soa,
                                                      int groups) {
  int64_t t = (int64_t)blockIdx.x * QXD_BLOCK + threadIdx.x;
  if (t >= 2 * (int64_t)g.Ve) return;
  int p = (int)(t / g.Ve), h = (int)(t % g.Ve);
  int x0, x1, x2, x3;
  geo_decode(g, p, h, x0, x1, x2, x3);
  int64_t s = (int64_t)x3 + (int64_t)g.Le3 * ((int64_t)x2 + (int64_t)g.Le2 * ((int64_t)x1 + (int64_t)g.Le1 * x0));
  cx<T> v[12];
  sp_load(soa + (size_t)p * groups * g.Ve, g.Ve, h, v);
#pragma unroll
  for (int c = 0; c < 12; ++c) aos[s * 12 + c] = make_double2((double)v[c].re, (double)v[c].im);
}

template <class SPT, class T>
__global__ __launch_bounds__(QXD_BLOCK) void k_pack2(Geo g, SPT* __restrict__ soa, const double2* __restrict__ aos,
                                                     int groups) {
  int64_t t = (int64_t)blockIdx.x * QXD_BLOCK + threadIdx.x;
  if (t >= 2 * (int64_t)g.Ve) return;
  int p = (int)(t / g.Ve), h = (int)(t % g.Ve);
  int x0, x1, x2, x3;
  geo_decode(g, p, h, x0, x1, x2, x3);
  int64_t s = (int64_t)x3 + (int64_t)g.Le3 * ((int64_t)x2 + (int64_t)g.Le2 * ((int64_t)x1 + (int64_t)g.Le1 * x0));
  cx<T> v[12];
#pragma unroll
  for (int c = 0; c < 12; ++c) {
    double2 a = aos[s * 12 + c];
    v[c] = mk((T)a.x, (T)a.y);
  }
  sp_store(soa + (size_t)p * groups * g.Ve, g.Ve, h, v);
}

// ---------------------------------------------------------------------------
// host side

static int groups_of(qxd_prec p) { return p == QXD_F64 ? 12 : p == QXD_F32 ? 6 : 3; }

static size_t half_bytes(const qxd_handle* h, qxd_prec p) { return (size_t)groups_of(p) * 16 * h->Ve; }

static qxd_status ensure_t(qxd_handle* h, qxd_prec p) {
  void** t = p == QXD_F64 ? (void**)&h->t64 : p == QXD_F32 ? (void**)&h->t32 : (void**)&h->t16;
  if (!*t && !dev_alloc(t, half_bytes(h, p))) return QXD_ENOMEM;
  return QXD_OK;
}


// Pass-by-pass order of the Schur launches.  Both passes are memory bound and
// pass 2 reads back t_o and psi_e, which pass 1 wrote and read.  Run over the
// whole lattice, pass 1 moves several times the last-level cache between the
// two, so pass 2 finds neither there.  Instead the time slices are taken in
// chunks of C: pass 1 on chunk k, then pass 2 on the slices whose three t_o
// time neighbours are now all written (chunk k shifted back by one slice).
// Time is periodic: the first chunk starts at the last slice, so that the
// pass 2 after the last chunk covers the remaining C + 2 slices in one launch.
// Every site is computed exactly as in the two-launch order (bit-identical
// results, partial sums indexed by tile), and pass 2 reads t_o and psi_e while
// they are still in the 256 MB last-level cache.  C is the largest divisor of the time
// extent (at most half of it) for which the t_o and psi_e of a chunk take at
// most 256 MB, used when it is at least 8 slices; otherwise (and where the
// slices are not whole tiles) two plain launches.  Measured at 64x64x32x32
// (128 tiles a slice): FP64 D_hat 1.786 ms in two launches, 1.688 ms with chunks
// of 16 slices (8 launches), 1.737 with 8; FP32 0.899 -> 0.862 (32 slices);
// bf16 storage 0.564 -> 0.556 (32 slices).  At 128x128x64x64 a slice holds
// 100 MB per array and chunks of 2, 4 or 8 slices are slower (FP64 27.6 ms ->
// 29.1-30.0).  Running pass 2 of a chunk on a side stream beside pass 1 of the
// next was slower as well (1.772 ms).
static int schur_slices(const qxd_handle* h, qxd_prec p) {
  const int64_t S = h->Ve / h->geo.Le0;  // half sites per time slice
  if (S % QXD_BLOCK) return 0;
  int c = h->slices_env;
  if (c < 0) {
    const double per_slice = (double)S * 2 * (p == QXD_F64 ? 192 : p == QXD_F32 ? 96 : 48);
    c = (int)(256e6 / per_slice);
  }
  if (c > h->geo.Le0 / 2) c = h->geo.Le0 / 2;
  while (c >= 2 && h->geo.Le0 % c) --c;
  if (h->slices_env < 0 && c < 8) return 0;
  return c >= 2 ? c : 0;
}

template <class T, class SPT, class LKT, class CLT>
static void launch_schur(qxd_handle* h, int dagger, SPT* out, const SPT* in, SPT* t, const LKT* V, const CLT* He,
                         const CLT* Hi, double* norm_slot, int slices, hipStream_t s) {
  const size_t lk_half = (size_t)4 * 9 * h->Ve;
  const LKT* Ve_l = V;
  const LKT* Vo_l = V + lk_half;
  const int G = div_up(h->Ve, QXD_BLOCK);
  Geo g = h->geo;
  auto pass1 = [&](int tile0, int n) {
    g.tile0 = tile0;
    if (dagger)
      hipLaunchKernelGGL((k_schur1<T, SPT, LKT, CLT, true>), dim3(n), dim3(QXD_BLOCK), 0, s, g, in, t, Ve_l, Vo_l, Hi);
    else
      hipLaunchKernelGGL((k_schur1<T, SPT, LKT, CLT, false>), dim3(n), dim3(QXD_BLOCK), 0, s, g, in, t, Ve_l, Vo_l, Hi);
  };
  auto pass2 = [&](int tile0, int n) {
    g.tile0 = tile0;
    if (n <= 0) return;
    if (norm_slot) {
      if (dagger)
        hipLaunchKernelGGL((k_schur2<T, SPT, LKT, CLT, true, true>), dim3(n), dim3(QXD_BLOCK), 0, s, g, t, in, out,
                           Ve_l, Vo_l, He, h->partial);
      else
        hipLaunchKernelGGL((k_schur2<T, SPT, LKT, CLT, false, true>), dim3(n), dim3(QXD_BLOCK), 0, s, g, t, in, out,
                           Ve_l, Vo_l, He, h->partial);
    } else {
      if (dagger)
        hipLaunchKernelGGL((k_schur2<T, SPT, LKT, CLT, true, false>), dim3(n), dim3(QXD_BLOCK), 0, s, g, t, in, out,
                           Ve_l, Vo_l, He, nullptr);
      else
        hipLaunchKernelGGL((k_schur2<T, SPT, LKT, CLT, false, false>), dim3(n), dim3(QXD_BLOCK), 0, s, g, t, in, out,
                           Ve_l, Vo_l, He, nullptr);
    }
  };
  if (slices == 0) {
    g.ntile = 0;
    pass1(0, G);
    pass2(0, G);
  } else {
    const int T1 = (int)(h->Ve / h->geo.Le0 / QXD_BLOCK);  // tiles per time slice
    const int C = slices, nchunk = h->geo.Le0 / slices;
    g.ntile = G;
    // chunk k: slices kC - 1 .. (k+1)C - 2 (chunk 0 starts at the last slice);
    // after it, pass 2 on kC - 2 .. (k+1)C - 3, after the last on the rest
    pass1((h->geo.Le0 - 1) * T1, C * T1);
    pass2(0, (C - 2) * T1);
    for (int k = 1; k < nchunk; ++k) {
      pass1((k * C - 1) * T1, C * T1);
      pass2((k * C - 2) * T1, (k + 1 < nchunk ? C : C + 2) * T1);
    }
  }
  if (norm_slot) launch_final_sum(h->partial, G, 1, G, norm_slot, s);
}

// Workgroup walk for the Schur passes (site_tile): windows of K tiles per XCD.
// Measured with non-temporal output stores, the same K for every precision:
// with 128 tiles per time slice (64x64x32x32) K = 8 is best (FP64 1.78 ms
// against 1.80 at K = 16), with 1024 (128x128x64x64) K = 16 (27.3-27.6 ms
// against 28.1).
static int walk_chunk(const qxd_handle* h, qxd_prec p) {
  (void)p;
  if (h->tchunk_env) return h->geo.tchunk;
  const int64_t tiles_per_slice = (int64_t)h->geo.L3h * h->geo.Le2 * h->geo.Le1 / QXD_BLOCK;
  return tiles_per_slice >= 512 ? 16 : 8;
}

qxd_status qxd_schur_apply(qxd_handle* h, qxd_prec p, int dagger, void* out_e, const void* in_e, double* norm_slot,
                           hipStream_t s) {
  if (!h->has_inverse) return QXD_ESTATE;
  QXD_TRY(ensure_t(h, p));
  if (p != QXD_F64) QXD_TRY(ensure_copies(h, (p == QXD_F32 ? CP_V32 : CP_V16) | CP_HE32 | CP_HI32, s));
  h->geo.tchunk = walk_chunk(h, p);
  switch (p) {
    case QXD_F64:
      launch_schur<double>(h, dagger, (double2*)out_e, (const double2*)in_e, h->t64, (const double2*)h->V64,
                           (const double2*)h->He64, (const double2*)h->Hi64, norm_slot, schur_slices(h, p), s);
      break;
    case QXD_F32:
      launch_schur<float>(h, dagger, (float4*)out_e, (const float4*)in_e, h->t32, (const float2*)h->V32,
                          (const float4*)h->He32, (const float4*)h->Hi32, norm_slot, schur_slices(h, p), s);
      break;
    case QXD_BF16:
      launch_schur<float>(h, dagger, (uint4*)out_e, (const uint4*)in_e, h->t16, (const uint32_t*)h->V16,
                          (const float4*)h->He32, (const float4*)h->Hi32, norm_slot, schur_slices(h, p), s);
      break;
    default:
      return QXD_EINVAL;
  }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

// BF16 links with FP32 spinors (the inner operator of the BF16 solver mode)
qxd_status qxd_schur_apply_mixed(qxd_handle* h, int dagger, float4* out_e, const float4* in_e, double* norm_slot,
                                 hipStream_t s) {
  if (!h->has_inverse) return QXD_ESTATE;
  QXD_TRY(ensure_t(h, QXD_F32));
  QXD_TRY(ensure_copies(h, CP_V16 | CP_HE32 | CP_HI32, s));
  h->geo.tchunk = walk_chunk(h, QXD_F32);
  launch_schur<float>(h, dagger, out_e, in_e, h->t32, (const uint32_t*)h->V16, (const float4*)h->He32,
                      (const float4*)h->Hi32, norm_slot, schur_slices(h, QXD_F32), s);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_dw_eo_schur(qxd_handle* h, qxd_prec p, int dagger, void* out_e, const void* in_e,
                                      void* stream) {
  if (!h || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  if (p != QXD_F64 && p != QXD_F32 && p != QXD_BF16) return QXD_EINVAL;
  return qxd_schur_apply(h, p, dagger ? 1 : 0, out_e, in_e, nullptr, as_stream(stream));
}

// ---------------------------------------------------------------------------
// D_hat without allocation.  The odd-site workspace t_o of the two passes lives
// in a static device array instead of a handle buffer allocated on first use,
// so the call allocates nothing.  In host code `scratch` names the host-side
// shadow of the array, not device memory: its device address (one copy per
// GPU) is looked up once per device by scratch_resolve and only that address
// is ever handed to a kernel.  Nothing in the array must start at zero (pass 1
// writes every odd site before pass 2 reads it); calls that overlap on one GPU
// share the array and race.

static __device__ __align__(256) unsigned char scratch[QXD_NOALLOC_SCRATCH_BYTES];

#define QXD_MAX_DEVICES 64
static void* g_scratch_dev[QXD_MAX_DEVICES];
static std::mutex g_scratch_mu;

qxd_status scratch_resolve(int device) {
  if (device < 0 || device >= QXD_MAX_DEVICES) return QXD_EINVAL;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_dev[device]) return QXD_OK;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return QXD_EHIP;
  g_scratch_dev[device] = ptr;
  return QXD_OK;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return device >= 0 && device < QXD_MAX_DEVICES ? g_scratch_dev[device] : nullptr;
}

extern "C" qxd_status qxd_dw_eo_schur_noalloc(qxd_handle* h, qxd_prec p, int dagger, void* out_e, const void* in_e,
                                              void* stream) {
  if (!h || !out_e || !in_e || out_e == in_e) return QXD_EINVAL;
  if (p != QXD_F64 && p != QXD_F32 && p != QXD_BF16) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  if (half_bytes(h, p) > (size_t)QXD_NOALLOC_SCRATCH_BYTES) return QXD_ESCRATCH;
  // the FP32 / bf16 operator copies are made by an allocating call (not here)
  const unsigned need = p == QXD_F64 ? 0u : (p == QXD_F32 ? CP_V32 : CP_V16) | CP_HE32 | CP_HI32;
  if ((h->copies & need) != need) return QXD_ESTATE;
  int dev = -1;
  QXD_HIP(hipGetDevice(&dev));
  if (dev != h->device) return QXD_EINVAL;
  void* t = scratch_of(dev);
  if (!t) return QXD_ESTATE;  // qxd_create resolves it for the handle's device
  hipStream_t s = as_stream(stream);
  h->geo.tchunk = walk_chunk(h, p);
  switch (p) {
    case QXD_F64:
      launch_schur<double>(h, dagger ? 1 : 0, (double2*)out_e, (const double2*)in_e, (double2*)t,
                           (const double2*)h->V64, (const double2*)h->He64, (const double2*)h->Hi64, nullptr, schur_slices(h, p), s);
      break;
    case QXD_F32:
      launch_schur<float>(h, dagger ? 1 : 0, (float4*)out_e, (const float4*)in_e, (float4*)t, (const float2*)h->V32,
                          (const float4*)h->He32, (const float4*)h->Hi32, nullptr, schur_slices(h, p), s);
      break;
    default:
      launch_schur<float>(h, dagger ? 1 : 0, (uint4*)out_e, (const uint4*)in_e, (uint4*)t, (const uint32_t*)h->V16,
                          (const float4*)h->He32, (const float4*)h->Hi32, nullptr, schur_slices(h, p), s);
      break;
  }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

template <class T, class SPT, class LKT, class CLT>
static void launch_dw(qxd_handle* h, SPT* out, const SPT* in, const LKT* V, const CLT* He, const CLT* Ho, int groups,
                      hipStream_t s) {
  const size_t lk_half = (size_t)4 * 9 * h->Ve;
  const size_t sp_half = (size_t)groups * h->Ve;
  int G = div_up(h->Ve, QXD_BLOCK);
  hipLaunchKernelGGL((k_dw<T, SPT, LKT, CLT>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, 0, in, in + sp_half, out, V,
                     V + lk_half, He);
  hipLaunchKernelGGL((k_dw<T, SPT, LKT, CLT>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, 1, in + sp_half, in,
                     out + sp_half, V + lk_half, V, Ho);
}

extern "C" qxd_status qxd_dw_apply(qxd_handle* h, qxd_prec p, void* out, const void* in, void* stream) {
  if (!h || !out || !in || out == in) return QXD_EINVAL;
  if (!h->has_clover) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  switch (p) {
    case QXD_F64:
      launch_dw<double>(h, (double2*)out, (const double2*)in, (const double2*)h->V64, (const double2*)h->He64,
                        (const double2*)h->Ho64, 12, s);
      break;
    case QXD_F32:
    case QXD_BF16:
      QXD_TRY(ensure_copies(h, (p == QXD_F32 ? CP_V32 : CP_V16) | CP_HE32 | CP_HO32, s));
      if (p == QXD_F32)
        launch_dw<float>(h, (float4*)out, (const float4*)in, (const float2*)h->V32, (const float4*)h->He32,
                         (const float4*)h->Ho32, 6, s);
      else
        launch_dw<float>(h, (uint4*)out, (const uint4*)in, (const uint32_t*)h->V16, (const float4*)h->He32,
                         (const float4*)h->Ho32, 3, s);
      break;
    default:
      return QXD_EINVAL;
  }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_eo_source(qxd_handle* h, void* bhat_e, const void* b, void* stream) {
  if (!h || !bhat_e || !b) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  QXD_TRY(ensure_t(h, QXD_F64));
  hipStream_t s = as_stream(stream);
  const double2* bb = (const double2*)b;
  const size_t sp_half = (size_t)12 * h->Ve, lk_half = (size_t)4 * 9 * h->Ve;
  int G = div_up(h->Ve, QXD_BLOCK);
  // t_o = H_o^-1 b_o ;  bhat_e = b_e + (1/2) hop(t_o)
  hipLaunchKernelGGL(k_clov, dim3(G), dim3(QXD_BLOCK), 0, s, (int)h->Ve, bb + sp_half, h->t64, (const double2*)h->Hi64);
  hipLaunchKernelGGL(k_hop_add<false>, dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, 0, h->t64, bb, (double2*)bhat_e,
                     h->V64, h->V64 + lk_half, nullptr, 0.5);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_eo_reconstruct(qxd_handle* h, void* x, const void* x_e, const void* b, void* stream) {
  if (!h || !x || !x_e || !b) return QXD_EINVAL;
  if (!h->has_inverse) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  const size_t sp_half = (size_t)12 * h->Ve, lk_half = (size_t)4 * 9 * h->Ve;
  double2* xx = (double2*)x;
  if (x_e != x) QXD_HIP(hipMemcpyAsync(xx, x_e, sp_half * sizeof(double2), hipMemcpyDeviceToDevice, s));
  int G = div_up(h->Ve, QXD_BLOCK);
  // x_o = H_o^-1 (b_o + (1/2) hop(x_e))
  hipLaunchKernelGGL(k_hop_add<true>, dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, 1, (const double2*)xx,
                     (const double2*)b + sp_half, xx + sp_half, h->V64 + lk_half, h->V64, (const double2*)h->Hi64,
                     0.5);
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_pack(qxd_handle* h, qxd_prec p, void* soa, const double* aos, void* stream) {
  if (!h || !soa || !aos) return QXD_EINVAL;
  hipStream_t s = as_stream(stream);
  int G = div_up(2 * h->Ve, QXD_BLOCK);
  const double2* a = (const double2*)aos;
  switch (p) {
    case QXD_F64: hipLaunchKernelGGL((k_pack2<double2, double>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, (double2*)soa, a, 12); break;
    case QXD_F32: hipLaunchKernelGGL((k_pack2<float4, float>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, (float4*)soa, a, 6); break;
    case QXD_BF16: hipLaunchKernelGGL((k_pack2<uint4, float>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, (uint4*)soa, a, 3); break;
    default: return QXD_EINVAL;
  }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}

extern "C" qxd_status qxd_unpack(qxd_handle* h, qxd_prec p, double* aos, const void* soa, void* stream) {
  if (!h || !soa || !aos) return QXD_EINVAL;
  hipStream_t s = as_stream(stream);
  int G = div_up(2 * h->Ve, QXD_BLOCK);
  double2* a = (double2*)aos;
  switch (p) {
    case QXD_F64: hipLaunchKernelGGL((k_unpack<double2, double>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, a, (const double2*)soa, 12); break;
    case QXD_F32: hipLaunchKernelGGL((k_unpack<float4, float>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, a, (const float4*)soa, 6); break;
    case QXD_BF16: hipLaunchKernelGGL((k_unpack<uint4, float>), dim3(G), dim3(QXD_BLOCK), 0, s, h->geo, a, (const uint4*)soa, 3); break;
    default: return QXD_EINVAL;
  }
  QXD_HIP(hipGetLastError());
  return QXD_OK;
}
