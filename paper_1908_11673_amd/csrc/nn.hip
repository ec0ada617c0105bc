// Network preconditioner (filled in below the Dirac path).
#include "qxd_internal.hpp"

struct qxd_nn {
  qxd_handle* h;
};

qxd_status nn_apply_internal(qxd_handle*, qxd_nn*, float4*, const float4*, hipStream_t) { return QXD_EINVAL; }

extern "C" qxd_status qxd_nn_create(qxd_handle*, qxd_nn**) { return QXD_EINVAL; }
extern "C" qxd_status qxd_nn_destroy(qxd_nn*) { return QXD_EINVAL; }
extern "C" qxd_status qxd_nn_set_weights(qxd_nn*, const float*) { return QXD_EINVAL; }
extern "C" qxd_status qxd_nn_get_weights(qxd_nn*, float*) { return QXD_EINVAL; }
extern "C" qxd_status qxd_nn_apply(qxd_handle*, qxd_nn*, void*, const void*, void*) { return QXD_EINVAL; }
extern "C" qxd_status qxd_nn_loss_grad(qxd_handle*, qxd_nn*, const void*, const void*, int, double*, float*, void*) {
  return QXD_EINVAL;
}
extern "C" qxd_status qxd_nn_harvest(qxd_handle*, const void*, int, void*, void*, int*, void*) { return QXD_EINVAL; }
extern "C" qxd_status qxd_nn_train(qxd_handle*, qxd_nn*, const qxd_train_params*, const void*, const void*, int,
                                   qxd_train_stats*, void*) {
  return QXD_EINVAL;
}
