// Handle management of libqxd.
#include <cstdlib>
#include <cstring>
#include <new>

#include "qxd_internal.hpp"

extern "C" const char* qxd_status_string(qxd_status s) {
  switch (s) {
    case QXD_OK: return "QXD_OK";
    case QXD_EINVAL: return "QXD_EINVAL";
    case QXD_EGEOM: return "QXD_EGEOM";
    case QXD_ENOMEM: return "QXD_ENOMEM";
    case QXD_ESINGULAR: return "QXD_ESINGULAR";
    case QXD_ENAN: return "QXD_ENAN";
    case QXD_ENOCONV: return "QXD_ENOCONV";
    case QXD_EHIP: return "QXD_EHIP";
    case QXD_ESTATE: return "QXD_ESTATE";
    case QXD_ESCRATCH: return "QXD_ESCRATCH";
    case QXD_EIO: return "QXD_EIO";
  }
  return "QXD_UNKNOWN";
}

static void release(qxd_handle* h) {
  void* ptrs[] = {h->Uphys, h->Aphys, h->V64, h->V32, h->V16, h->He64, h->Ho64, h->Hi64, h->He32,
                  h->Ho32, h->Hi32, h->t64, h->t32, h->t16, h->partial, h->scal};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (int i = 0; i < 64; ++i)
    if (h->ws[i]) (void)hipFree(h->ws[i]);
  if (h->scal_host) (void)hipHostFree(h->scal_host);
}

extern "C" qxd_status qxd_create(const qxd_geom* g, qxd_handle** out) {
  if (!g || !out) return QXD_EINVAL;
  *out = nullptr;
  for (int m = 0; m < 4; ++m)
    if (g->L[m] < 2 || (g->L[m] & 1)) return QXD_EGEOM;
  if (g->cstar < 0 || g->cstar > 3) return QXD_EGEOM;
  int64_t Le1 = g->cstar >= 1 ? 2 * (int64_t)g->L[1] : g->L[1];
  int64_t V = (int64_t)g->L[0] * Le1 * g->L[2] * g->L[3];
  if (V >= ((int64_t)1 << 31)) return QXD_EGEOM;
  qxd_handle* h = new (std::nothrow) qxd_handle();
  if (!h) return QXD_ENOMEM;
  h->g = *g;
  h->V = V;
  h->Ve = V / 2;
  h->Vphys = (int64_t)g->L[0] * g->L[1] * g->L[2] * g->L[3];
  h->geo.Le0 = g->L[0];
  h->geo.Le1 = (int)Le1;
  h->geo.Le2 = g->L[2];
  h->geo.Le3 = g->L[3];
  h->geo.L1 = g->L[1];
  h->geo.cstar = g->cstar;
  h->geo.tanti = g->t_antiperiodic ? 1 : 0;
  h->geo.L3h = g->L[3] / 2;
  h->geo.Ve = (int)h->Ve;
  h->geo.tchunk = 8;
  if (const char* e = std::getenv("QXD_SCHUR_SLICES")) h->slices_env = std::atoi(e);
  if (const char* e = std::getenv("QXD_SCHUR_STORES")) h->geo.plain_st = std::strcmp(e, "plain") == 0;
  if (const char* e = std::getenv("QXD_TILE_CHUNK")) {
    h->geo.tchunk = std::atoi(e);
    h->tchunk_env = true;
  }
  if (hipGetDevice(&h->device) != hipSuccess || scratch_resolve(h->device) != QXD_OK) {
    delete h;
    return QXD_EHIP;
  }
  h->npartial = (size_t)QXD_MAX_PARTIAL;
  if ((size_t)div_up(h->Ve, 64) > h->npartial) h->npartial = (size_t)div_up(h->Ve, 64);
  if (!dev_alloc(&h->partial, h->npartial * sizeof(double)) ||
      !dev_alloc(&h->scal, QXD_NSCAL * sizeof(double)) ||
      hipHostMalloc(&h->scal_host, QXD_NSCAL * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();  // the failed allocation is reported as QXD_ENOMEM only
    release(h);
    delete h;
    return QXD_ENOMEM;
  }
  if (hipMemset(h->scal, 0, QXD_NSCAL * sizeof(double)) != hipSuccess) {
    release(h);
    delete h;
    return QXD_EHIP;
  }
  *out = h;
  return QXD_OK;
}

extern "C" qxd_status qxd_destroy(qxd_handle* h) {
  if (!h) return QXD_EINVAL;
  (void)hipDeviceSynchronize();
  release(h);
  delete h;
  return QXD_OK;
}

extern "C" qxd_status qxd_trim(qxd_handle* h) {
  if (!h) return QXD_EINVAL;
  QXD_HIP(hipDeviceSynchronize());
  void** ptrs[] = {reinterpret_cast<void**>(&h->Uphys), reinterpret_cast<void**>(&h->Aphys),
                   reinterpret_cast<void**>(&h->t64), reinterpret_cast<void**>(&h->t32),
                   reinterpret_cast<void**>(&h->t16)};
  for (void** p : ptrs) {
    if (*p) QXD_HIP(hipFree(*p));
    *p = nullptr;
  }
  for (int i = 0; i < 64; ++i) {
    if (h->ws[i]) QXD_HIP(hipFree(h->ws[i]));
    h->ws[i] = nullptr;
    h->ws_bytes[i] = 0;
  }
  release_copies(h);
  h->has_gauge = false;
  h->sap_gen = 0;  // its block-order copies went with the workspaces
  return QXD_OK;
}

void release_copies(qxd_handle* h, unsigned which) {
  const struct {
    unsigned bit;
    void** p;
  } cp[] = {{CP_V32, reinterpret_cast<void**>(&h->V32)}, {CP_V16, reinterpret_cast<void**>(&h->V16)},
            {CP_HE32, reinterpret_cast<void**>(&h->He32)}, {CP_HO32, reinterpret_cast<void**>(&h->Ho32)},
            {CP_HI32, reinterpret_cast<void**>(&h->Hi32)}};
  for (const auto& c : cp) {
    if (!(which & c.bit)) continue;
    if (*c.p) (void)hipFree(*c.p);
    *c.p = nullptr;
    h->copies &= ~c.bit;
  }
}

extern "C" qxd_status qxd_volume(const qxd_handle* h, int64_t* V, int64_t* Ve) {
  if (!h) return QXD_EINVAL;
  if (V) *V = h->V;
  if (Ve) *Ve = h->Ve;
  return QXD_OK;
}
