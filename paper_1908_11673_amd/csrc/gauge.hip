// Gauge preparation on the extended lattice (Sec. 2.1 and 2.3 of arXiv:1908.11673):
// the mirror half U(x + L1 e1) = U(x)*, A(x + L1 e1) = -A(x) is filled from the
// physical half on the fly, and the combined links V(x,mu) = U(x,mu) z(x,mu)^qhat
// with z = exp(i A) are written in the even-odd SoA layout in FP64; the FP32 and
// bf16 copies are made from them when first needed.
#include "qxd_internal.hpp"

// canonical physical site of extended coordinates, and whether x is on the mirror half
__device__ inline int64_t phys_site(const Geo& g, const int Lp[4], int x0, int x1, int x2, int x3, bool& mirror) {
  mirror = x1 >= Lp[1];
  int x1p = mirror ? x1 - Lp[1] : x1;
  return (int64_t)x3 + (int64_t)Lp[3] * ((int64_t)x2 + (int64_t)Lp[2] * ((int64_t)x1p + (int64_t)Lp[1] * x0));
}

struct PhysExt {
  int L[4];
  int64_t Vphys;
};

__global__ __launch_bounds__(QXD_BLOCK) void k_make_links(Geo g, PhysExt pe, const double2* __restrict__ U,
                                                           const double* __restrict__ A, int qhat,
                                                           double2* __restrict__ V64) {
  int64_t t = (int64_t)blockIdx.x * QXD_BLOCK + threadIdx.x;
  int64_t total = 2 * (int64_t)g.Ve * 4;
  if (t >= total) return;
  int h = (int)(t % g.Ve);
  int rest = (int)(t / g.Ve);
  int mu = rest & 3;
  int p = rest >> 2;
  int x0, x1, x2, x3;
  geo_decode(g, p, h, x0, x1, x2, x3);
  bool mirror;
  int64_t sp = phys_site(g, pe.L, x0, x1, x2, x3, mirror);
  double a = A[mu * pe.Vphys + sp];
  if (mirror) a = -a;
  double sn, cs;
  sincos((double)qhat * a, &sn, &cs);
  cx<double> z = mk(cs, sn);
  size_t Ve = g.Ve;
  size_t base = ((size_t)(p * 4 + mu) * 9) * Ve + h;
  for (int k = 0; k < 9; ++k) {
    double2 u = U[(mu * pe.Vphys + sp) * 9 + k];
    cx<double> uu = mk(u.x, mirror ? -u.y : u.y);
    cx<double> v = uu * z;
    V64[base + k * Ve] = make_double2(v.re, v.im);
  }
}

// FP32 and bf16 copies of the links (each entry rounded to FP32, then to bf16),
// regrouped so that a site's entries form 16-byte words; these stay aligned
// because Ve is a multiple of 8 (every extent of the lattice is even)
// entry k of link (parity, mu, h) goes to float2 lk32_index(Ve, k, h) of the
// 9 Ve of (parity, mu)
__global__ __launch_bounds__(QXD_BLOCK) void k_link_cast32(int64_t n, int64_t Ve, const double2* __restrict__ V64,
                                                            float2* __restrict__ V32) {
  int64_t t = (int64_t)blockIdx.x * QXD_BLOCK + threadIdx.x;
  if (t >= n) return;
  const int64_t h = t % Ve, r = t / Ve;
  const int k = (int)(r % 9);
  const int64_t pm = r / 9;
  double2 v = V64[t];
  V32[pm * 9 * Ve + lk32_index(Ve, k, h)] = make_float2((float)v.x, (float)v.y);
}
// entry k of link (parity, mu, h) goes to word 4 h + k (k < 4), 4 Ve + 4 h + k - 4
// (k < 8) or 8 Ve + h (k = 8) of the 9 Ve words of (parity, mu)
__global__ __launch_bounds__(QXD_BLOCK) void k_link_cast16(int64_t n, int64_t Ve, const double2* __restrict__ V64,
                                                            uint32_t* __restrict__ V16) {
  int64_t t = (int64_t)blockIdx.x * QXD_BLOCK + threadIdx.x;
  if (t >= n) return;
  const int64_t h = t % Ve, r = t / Ve;
  const int64_t k = r % 9, pm = r / 9;
  const int64_t dst = pm * 9 * Ve + (k < 4 ? 4 * h + k : k < 8 ? 4 * Ve + 4 * h + (k - 4) : 8 * Ve + h);
  double2 v = V64[t];
  V16[dst] = pack_bf16x2((float)v.x, (float)v.y);
}

qxd_status ensure_link_copies(qxd_handle* h, unsigned which, hipStream_t s) {
  const int64_t n = (int64_t)2 * 4 * 9 * h->Ve;
  if ((which & CP_V32) && !(h->copies & CP_V32)) {
    if (!h->has_flavour) return QXD_ESTATE;
    if (!h->V32 && !dev_alloc(&h->V32, n * sizeof(float2))) return QXD_ENOMEM;
    hipLaunchKernelGGL(k_link_cast32, dim3(div_up(n, QXD_BLOCK)), dim3(QXD_BLOCK), 0, s, n, (int64_t)h->Ve, h->V64,
                       h->V32);
    QXD_HIP(hipGetLastError());
    h->copies |= CP_V32;
  }
  if ((which & CP_V16) && !(h->copies & CP_V16)) {
    if (!h->has_flavour) return QXD_ESTATE;
    if (!h->V16 && !dev_alloc(&h->V16, n * sizeof(uint32_t))) return QXD_ENOMEM;
    hipLaunchKernelGGL(k_link_cast16, dim3(div_up(n, QXD_BLOCK)), dim3(QXD_BLOCK), 0, s, n, (int64_t)h->Ve, h->V64,
                       h->V16);
    QXD_HIP(hipGetLastError());
    h->copies |= CP_V16;
  }
  return QXD_OK;
}

extern "C" qxd_status qxd_set_gauge(qxd_handle* h, const double* U_phys, const double* A_phys, int on_device,
                                    void* stream) {
  if (!h || !U_phys || !A_phys) return QXD_EINVAL;
  hipStream_t s = as_stream(stream);
  size_t nU = (size_t)4 * h->Vphys * 18 * sizeof(double);
  size_t nA = (size_t)4 * h->Vphys * sizeof(double);
  if (!h->Uphys) {
    if (!dev_alloc(&h->Uphys, nU)) return QXD_ENOMEM;
    if (!dev_alloc(&h->Aphys, nA)) {
      (void)hipFree(h->Uphys);  // both or neither
      h->Uphys = nullptr;
      return QXD_ENOMEM;
    }
  }
  if (on_device) {
    QXD_HIP(hipMemcpyAsync(h->Uphys, U_phys, nU, hipMemcpyDeviceToDevice, s));
    QXD_HIP(hipMemcpyAsync(h->Aphys, A_phys, nA, hipMemcpyDeviceToDevice, s));
  } else {
    QXD_HIP(hipStreamSynchronize(s));
    QXD_HIP(hipMemcpy(h->Uphys, U_phys, nU, hipMemcpyHostToDevice));
    QXD_HIP(hipMemcpy(h->Aphys, A_phys, nA, hipMemcpyHostToDevice));
  }
  h->has_gauge = true;
  h->has_flavour = h->has_clover = h->has_inverse = false;
  return QXD_OK;
}

extern "C" qxd_status qxd_set_flavour(qxd_handle* h, const qxd_flavour* f, void* stream) {
  if (!h || !f) return QXD_EINVAL;
  if (!h->has_gauge) return QXD_ESTATE;
  if (!(f->kappa > 0.0) || !(f->invqel > 0.0)) return QXD_EINVAL;
  hipStream_t s = as_stream(stream);
  size_t nl = (size_t)2 * 4 * 9 * h->Ve;
  if (!h->V64 && !dev_alloc(&h->V64, nl * sizeof(double2))) return QXD_ENOMEM;
  h->copies = 0;
  PhysExt pe;
  for (int m = 0; m < 4; ++m) pe.L[m] = h->g.L[m];
  // without C* there is no mirror half: x1 never reaches L1
  pe.Vphys = h->Vphys;
  int64_t total = 2 * h->Ve * 4;
  hipLaunchKernelGGL(k_make_links, dim3(div_up(total, QXD_BLOCK)), dim3(QXD_BLOCK), 0, s, h->geo, pe,
                     reinterpret_cast<const double2*>(h->Uphys), h->Aphys, f->qhat, h->V64);
  QXD_HIP(hipGetLastError());
  h->fl = *f;
  h->has_flavour = true;
  h->has_clover = h->has_inverse = false;
  return QXD_OK;
}
