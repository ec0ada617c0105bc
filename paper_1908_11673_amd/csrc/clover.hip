// SW (clover) term and its odd-site inverse (Sec. 2.3 of arXiv:1908.11673).
//
// On every extended site the site-diagonal part of D is
//   1/(2 kappa) + sum_{mu<nu} (i/2) sigma_{mu nu} E_{mu nu},
//   E = su3csw F + u1csw qhat (i a) 1,  F = (Q - Q^+)/8 (four SU(3) clover leaves),
//   a = (1/4) sum of sin(plaquette angle) over the four U(1) plaquettes at x,
//       x-mu, x-nu, x-mu-nu (unit charge: the 1/q_el of the U(1) tensor cancels
//       against q = qhat q_el).
// In the chiral basis sigma_{0k} = diag(s_k, -s_k), sigma_{jk} = -eps_{jkl} diag(s_l, s_l),
// so the term is block diagonal: H_pm = 1/(2 kappa) + sum_l s_l (x) X_l^pm with
// X_l^pm = (i/2)(pm E_{0l} - E_{B_l}), B = ((2,3), (3,1), (1,2)).
#include "qxd_internal.hpp"

struct PhysExt2 {
  int L[4];
  int64_t Vphys;
};

__device__ inline void step_coords(const Geo& g, int x[4], int mu, int dir) {
  x[mu] += dir;
  int Le = mu == 0 ? g.Le0 : mu == 1 ? g.Le1 : mu == 2 ? g.Le2 : g.Le3;
  if (x[mu] < 0 || x[mu] >= Le) {
    x[mu] = x[mu] < 0 ? x[mu] + Le : x[mu] - Le;
    if (mu >= 2 && mu <= g.cstar) x[1] = geo_mirror_x1(g, x[1]);
  }
}

__device__ inline int64_t phys_of(const PhysExt2& pe, const int x[4], bool& mirror) {
  mirror = x[1] >= pe.L[1];
  int x1 = mirror ? x[1] - pe.L[1] : x[1];
  return (int64_t)x[3] + (int64_t)pe.L[3] * ((int64_t)x[2] + (int64_t)pe.L[2] * ((int64_t)x1 + (int64_t)pe.L[1] * x[0]));
}

struct M3 {
  cx<double> m[9];
};

__device__ inline M3 load_u(const PhysExt2& pe, const double2* __restrict__ U, const int x[4], int mu) {
  bool mir;
  int64_t s = phys_of(pe, x, mir);
  M3 r;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    double2 v = U[(mu * pe.Vphys + s) * 9 + k];
    r.m[k] = mk(v.x, mir ? -v.y : v.y);
  }
  return r;
}

__device__ inline double load_a(const PhysExt2& pe, const double* __restrict__ A, const int x[4], int mu) {
  bool mir;
  int64_t s = phys_of(pe, x, mir);
  double a = A[mu * pe.Vphys + s];
  return mir ? -a : a;
}

// a b, a^+ b, a b^+
__device__ inline M3 mm(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = a.m[3 * i] * b.m[j];
      s = s + a.m[3 * i + 1] * b.m[3 + j];
      s = s + a.m[3 * i + 2] * b.m[6 + j];
      r.m[3 * i + j] = s;
    }
  return r;
}
__device__ inline M3 mdm(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = cmul_conj(a.m[i], b.m[j]);
      s = s + cmul_conj(a.m[3 + i], b.m[3 + j]);
      s = s + cmul_conj(a.m[6 + i], b.m[6 + j]);
      r.m[3 * i + j] = s;
    }
  return r;
}
__device__ inline M3 mmd(const M3& a, const M3& b) {
  M3 r;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      cx<double> s = cmul_conj(b.m[3 * j], a.m[3 * i]);
      s = s + cmul_conj(b.m[3 * j + 1], a.m[3 * i + 1]);
      s = s + cmul_conj(b.m[3 * j + 2], a.m[3 * i + 2]);
      r.m[3 * i + j] = s;
    }
  return r;
}

// E_{mu nu}(x) = csw F + cu1 qhat (i a) 1 for one plane
__device__ inline M3 plane_tensor(const Geo& g, const PhysExt2& pe, const double2* U, const double* A, const int x[4],
                                  int mu, int nu, double csw, double cq) {
  int xpm[4], xpn[4], xmm[4], xmn[4], xmmpn[4], xmmmn[4], xmnpm[4];
  for (int i = 0; i < 4; ++i) xpm[i] = xpn[i] = xmm[i] = xmn[i] = x[i];
  step_coords(g, xpm, mu, +1);
  step_coords(g, xpn, nu, +1);
  step_coords(g, xmm, mu, -1);
  step_coords(g, xmn, nu, -1);
  for (int i = 0; i < 4; ++i) xmmpn[i] = xmmmn[i] = xmm[i];
  step_coords(g, xmmpn, nu, +1);
  step_coords(g, xmmmn, nu, -1);
  for (int i = 0; i < 4; ++i) xmnpm[i] = xmn[i];
  step_coords(g, xmnpm, mu, +1);

  M3 Q, t;
  // leaf at corner x: U(x,mu) U(x+mu,nu) U(x+nu,mu)^+ U(x,nu)^+
  t = mm(load_u(pe, U, x, mu), load_u(pe, U, xpm, nu));
  t = mmd(t, load_u(pe, U, xpn, mu));
  Q = mmd(t, load_u(pe, U, x, nu));
  // leaf at corner x-mu: U(x,nu) U(x-mu+nu,mu)^+ U(x-mu,nu)^+ U(x-mu,mu)
  t = mmd(load_u(pe, U, x, nu), load_u(pe, U, xmmpn, mu));
  t = mmd(t, load_u(pe, U, xmm, nu));
  t = mm(t, load_u(pe, U, xmm, mu));
  for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + t.m[k];
  // leaf at corner x-mu-nu: U(x-mu,mu)^+ U(x-mu-nu,nu)^+ U(x-mu-nu,mu) U(x-nu,nu)
  M3 a = load_u(pe, U, xmm, mu), b = load_u(pe, U, xmmmn, nu);
  // a^+ b^+ = (b a)^+
  M3 ba = mm(b, a);
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) t.m[3 * i + j] = conj(ba.m[3 * j + i]);
  t = mm(t, load_u(pe, U, xmmmn, mu));
  t = mm(t, load_u(pe, U, xmn, nu));
  for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + t.m[k];
  // leaf at corner x-nu: U(x-nu,nu)^+ U(x-nu,mu) U(x-nu+mu,nu) U(x,mu)^+
  t = mdm(load_u(pe, U, xmn, nu), load_u(pe, U, xmn, mu));
  t = mm(t, load_u(pe, U, xmnpm, nu));
  t = mmd(t, load_u(pe, U, x, mu));
  for (int k = 0; k < 9; ++k) Q.m[k] = Q.m[k] + t.m[k];

  // U(1): plaquette angles at the four corners
  auto angle = [&](const int y[4]) {
    int ym[4], yn[4];
    for (int i = 0; i < 4; ++i) ym[i] = yn[i] = y[i];
    step_coords(g, ym, mu, +1);
    step_coords(g, yn, nu, +1);
    return load_a(pe, A, y, mu) + load_a(pe, A, ym, nu) - load_a(pe, A, yn, mu) - load_a(pe, A, y, nu);
  };
  double a4 = 0.25 * (sin(angle(x)) + sin(angle(xmm)) + sin(angle(xmn)) + sin(angle(xmmmn)));

  M3 E;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cx<double> f = 0.125 * (Q.m[3 * i + j] - conj(Q.m[3 * j + i]));
      E.m[3 * i + j] = csw * f;
    }
  for (int i = 0; i < 3; ++i) E.m[4 * i].im += cq * a4;
  return E;
}

__global__ __launch_bounds__(128) void k_clover_build(Geo g, PhysExt2 pe, const double2* __restrict__ U,
                                                      const double* __restrict__ A, double csw, double cq,
                                                      double diag, double2* __restrict__ He,
                                                      double2* __restrict__ Ho) {
  int64_t t = (int64_t)blockIdx.x * 128 + threadIdx.x;
  if (t >= 2 * (int64_t)g.Ve) return;
  int p = (int)(t / g.Ve);
  int h = (int)(t % g.Ve);
  int x[4];
  geo_decode(g, p, h, x[0], x[1], x[2], x[3]);
  // planes: 01 02 03 12 13 23
  M3 E01 = plane_tensor(g, pe, U, A, x, 0, 1, csw, cq);
  M3 E02 = plane_tensor(g, pe, U, A, x, 0, 2, csw, cq);
  M3 E03 = plane_tensor(g, pe, U, A, x, 0, 3, csw, cq);
  M3 E12 = plane_tensor(g, pe, U, A, x, 1, 2, csw, cq);
  M3 E13 = plane_tensor(g, pe, U, A, x, 1, 3, csw, cq);
  M3 E23 = plane_tensor(g, pe, U, A, x, 2, 3, csw, cq);
  double2* out = p == 0 ? He : Ho;
  size_t Ve = g.Ve;
  for (int b = 0; b < 2; ++b) {
    double sg = b == 0 ? 1.0 : -1.0;
    // X_l = (i/2)(sg E_0l - E_Bl);  E_B2 = E_31 = -E_13
    M3 X1, X2, X3;
    for (int k = 0; k < 9; ++k) {
      cx<double> e1 = sg * E01.m[k] - E23.m[k];
      cx<double> e2 = sg * E02.m[k] + E13.m[k];
      cx<double> e3 = sg * E03.m[k] - E12.m[k];
      X1.m[k] = 0.5 * ti(e1);
      X2.m[k] = 0.5 * ti(e2);
      X3.m[k] = 0.5 * ti(e3);
    }
    double r[36];
    for (int a = 0; a < 3; ++a) {
      r[a] = diag + X3.m[4 * a].re;
      r[3 + a] = diag - X3.m[4 * a].re;
    }
    for (int i = 0; i < 6; ++i)
      for (int j = i + 1; j < 6; ++j) {
        int si = i / 3, ai = i % 3, sj = j / 3, aj = j % 3;
        cx<double> v;
        if (si == 0 && sj == 0) v = X3.m[3 * ai + aj];
        else if (si == 1 && sj == 1) v = -X3.m[3 * ai + aj];
        else v = X1.m[3 * ai + aj] - ti(X2.m[3 * ai + aj]);
        int o = herm6_off(i, j);
        r[o] = v.re;
        r[o + 1] = v.im;
      }
    for (int k = 0; k < 18; ++k) out[(18 * b + k) * Ve + h] = make_double2(r[2 * k], r[2 * k + 1]);
  }
}

// ---------------------------------------------------------------------------
// 6x6 inversion by Gauss-Jordan elimination with partial pivoting (largest
// |a|, lowest row on ties), fully unrolled so that row swaps are selects.

struct InvStats {
  unsigned long long* min_pivot_bits;  // positive doubles order as their bit patterns
  unsigned long long* max_norm_bits;
  unsigned long long* n_singular;
};

__device__ inline void invert6(const double* r, double* out, double& minpiv, double& maxabs) {
  cx<double> A[6][6], B[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j < 6; ++j) B[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
    A[i][i] = mk(r[i], 0.0);
  }
  maxabs = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    maxabs = fmax(maxabs, fabs(r[i]));
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      int o = herm6_off(i, j);
      A[i][j] = mk(r[o], r[o + 1]);
      A[j][i] = mk(r[o], -r[o + 1]);
      maxabs = fmax(maxabs, sqrt(r[o] * r[o] + r[o + 1] * r[o + 1]));
    }
  }
  minpiv = 1e300;
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    int p = k;
    double best = norm2(A[k][k]);
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      double v = norm2(A[i][k]);
      if (v > best) { best = v; p = i; }
    }
#pragma unroll
    for (int i = k + 1; i < 6; ++i) {
      bool sw = (p == i);
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        cx<double> a = A[k][j], b = A[i][j], c = B[k][j], d = B[i][j];
        A[k][j] = sw ? b : a;
        A[i][j] = sw ? a : b;
        B[k][j] = sw ? d : c;
        B[i][j] = sw ? c : d;
      }
    }
    minpiv = fmin(minpiv, sqrt(best));
    cx<double> piv = A[k][k];
    double den = 1.0 / norm2(piv);
    cx<double> inv = mk(piv.re * den, -piv.im * den);
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      A[k][j] = inv * A[k][j];
      B[k][j] = inv * B[k][j];
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i == k) continue;
      cx<double> f = A[i][k];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        A[i][j] = A[i][j] - f * A[k][j];
        B[i][j] = B[i][j] - f * B[k][j];
      }
    }
  }
  // pack the (Hermitian) inverse, symmetrised
#pragma unroll
  for (int i = 0; i < 6; ++i) out[i] = B[i][i].re;
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      int o = herm6_off(i, j);
      out[o] = 0.5 * (B[i][j].re + B[j][i].re);
      out[o + 1] = 0.5 * (B[i][j].im - B[j][i].im);
    }
}

__device__ inline double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

__global__ __launch_bounds__(64) void k_clover_invert(int Ve, const double2* __restrict__ Ho,
                                                      double2* __restrict__ Hi, InvStats st) {
  int h = blockIdx.x * 64 + threadIdx.x;
  double mp = 1e300, mx = 0.0;
  unsigned long long nsing = 0;
  if (h < Ve) {
    size_t sVe = Ve;
    for (int b = 0; b < 2; ++b) {
      double r[36], o[36];
      for (int k = 0; k < 18; ++k) {
        double2 v = Ho[(18 * b + k) * sVe + h];
        r[2 * k] = v.x;
        r[2 * k + 1] = v.y;
      }
      double piv, nrm;
      invert6(r, o, piv, nrm);
      mp = fmin(mp, piv);
      mx = fmax(mx, nrm);
      if (!(piv >= 1e-14 * nrm)) ++nsing;  // also counts NaN
      for (int k = 0; k < 18; ++k) Hi[(18 * b + k) * sVe + h] = make_double2(o[2 * k], o[2 * k + 1]);
    }
  }
  mp = wave_min(mp);
  mx = wave_max(mx);
  for (int off = 32; off > 0; off >>= 1) nsing += __shfl_xor(nsing, off);
  if (threadIdx.x == 0) {
    atomicMin(st.min_pivot_bits, (unsigned long long)__double_as_longlong(mp));
    atomicMax(st.max_norm_bits, (unsigned long long)__double_as_longlong(mx));
    if (nsing) atomicAdd(st.n_singular, nsing);
  }
}

// FP64 [36][Ve] double2 -> FP32 [18][Ve] float4
__global__ __launch_bounds__(QXD_BLOCK) void k_clover_cast(int Ve, const double2* __restrict__ in,
                                                           float4* __restrict__ out) {
  int64_t t = (int64_t)blockIdx.x * QXD_BLOCK + threadIdx.x;
  if (t >= (int64_t)18 * Ve) return;
  int k = (int)(t / Ve), h = (int)(t % Ve);
  size_t sVe = Ve;
  double2 a = in[(2 * k) * sVe + h], b = in[(2 * k + 1) * sVe + h];
  out[k * sVe + h] = make_float4((float)a.x, (float)a.y, (float)b.x, (float)b.y);
}

static qxd_status alloc_clover(qxd_handle* h) {
  if (h->He64) return QXD_OK;
  size_t n64 = (size_t)36 * h->Ve * sizeof(double2);
  if (!dev_alloc(&h->He64, n64) || !dev_alloc(&h->Ho64, n64) || !dev_alloc(&h->Hi64, n64)) {
    for (double2** p : {&h->He64, &h->Ho64, &h->Hi64}) {  // all or none, so that the next call allocates again
      if (*p) (void)hipFree(*p);
      *p = nullptr;
    }
    return QXD_ENOMEM;
  }
  return QXD_OK;
}

qxd_status ensure_link_copies(qxd_handle* h, unsigned which, hipStream_t s);  // gauge.hip

qxd_status ensure_copies(qxd_handle* h, unsigned which, hipStream_t s) {
  QXD_TRY(ensure_link_copies(h, which, s));
  const size_t n32 = (size_t)18 * h->Ve * sizeof(float4);
  const int g18 = div_up(18 * h->Ve, QXD_BLOCK);
  struct {
    unsigned bit;
    bool ready;
    double2* src;
    float4** dst;
  } cl[3] = {{CP_HE32, h->has_clover, h->He64, &h->He32},
             {CP_HO32, h->has_clover, h->Ho64, &h->Ho32},
             {CP_HI32, h->has_inverse, h->Hi64, &h->Hi32}};
  for (auto& c : cl) {
    if (!(which & c.bit) || (h->copies & c.bit)) continue;
    if (!c.ready) return QXD_ESTATE;
    if (!*c.dst && !dev_alloc(c.dst, n32)) return QXD_ENOMEM;
    hipLaunchKernelGGL(k_clover_cast, dim3(g18), dim3(QXD_BLOCK), 0, s, (int)h->Ve, c.src, *c.dst);
    QXD_HIP(hipGetLastError());
    h->copies |= c.bit;
  }
  return QXD_OK;
}

extern "C" qxd_status qxd_clover_build(qxd_handle* h, void* stream) {
  if (!h) return QXD_EINVAL;
  if (!h->has_flavour || !h->Uphys) return QXD_ESTATE;
  QXD_TRY(alloc_clover(h));
  hipStream_t s = as_stream(stream);
  PhysExt2 pe;
  for (int m = 0; m < 4; ++m) pe.L[m] = h->g.L[m];
  pe.Vphys = h->Vphys;
  double cq = h->fl.u1csw * (double)h->fl.qhat;
  double diag = 1.0 / (2.0 * h->fl.kappa);
  hipLaunchKernelGGL(k_clover_build, dim3(div_up(2 * h->Ve, 128)), dim3(128), 0, s, h->geo, pe,
                     reinterpret_cast<const double2*>(h->Uphys), h->Aphys, h->fl.su3csw, cq, diag, h->He64,
                     h->Ho64);
  QXD_HIP(hipGetLastError());
  h->has_clover = true;
  h->has_inverse = false;
  h->copies &= ~(CP_HE32 | CP_HO32 | CP_HI32);
  return QXD_OK;
}

extern "C" qxd_status qxd_clover_invert(qxd_handle* h, qxd_clover_stats* stats, void* stream) {
  if (!h) return QXD_EINVAL;
  if (!h->has_clover) return QXD_ESTATE;
  hipStream_t s = as_stream(stream);
  unsigned long long* d = reinterpret_cast<unsigned long long*>(h->scal + QXD_NSCAL - 8);
  unsigned long long init[3] = {(unsigned long long)__builtin_bit_cast(long long, 1e300), 0ull, 0ull};
  QXD_HIP(hipMemcpyAsync(d, init, sizeof(init), hipMemcpyHostToDevice, s));
  InvStats st{d, d + 1, d + 2};
  hipLaunchKernelGGL(k_clover_invert, dim3(div_up(h->Ve, 64)), dim3(64), 0, s, (int)h->Ve, h->Ho64, h->Hi64, st);
  QXD_HIP(hipGetLastError());
  h->copies &= ~CP_HI32;
  unsigned long long res[3];
  QXD_HIP(hipMemcpyAsync(res, d, sizeof(res), hipMemcpyDeviceToHost, s));
  QXD_HIP(hipStreamSynchronize(s));
  double mp = __builtin_bit_cast(double, (long long)res[0]);
  double mx = __builtin_bit_cast(double, (long long)res[1]);
  if (stats) {
    stats->min_pivot = mp;
    stats->max_norm = mx;
    stats->n_singular = (int64_t)res[2];
  }
  if (res[2] != 0) return QXD_ESINGULAR;
  h->has_inverse = true;
  ++h->setup_gen;
  return QXD_OK;
}
