"""Training driver of the learned preconditioner (orchestration of C ABI calls).

The network is local and translation invariant, so weights trained on one
lattice apply to any lattice with the same field statistics.  Training pairs
(r, e) belong to a gauge field: the residual-norm loss applies that field's
D_hat, so pairs are harvested and trained field by field (one qxd_nn_train
call per field and pass; the Adam state lives in the network).
"""
from __future__ import annotations

import time

import numpy as np

from . import (Lattice, qxd_clover_build, qxd_clover_invert, qxd_nn_create, qxd_nn_destroy,
               qxd_nn_get_weights, qxd_nn_harvest, qxd_nn_set_skip, qxd_nn_set_weights, qxd_nn_train,
               qxd_set_flavour, qxd_set_gauge, train_params)

SHAPES = [(24, 32), (32, 32), (32, 24)]


def initial_weights(seed: int, last_scale: float = 0.05) -> np.ndarray:
    """He-scaled Gaussian weights; the last layer starts near zero, so the
    network starts as M(r) = skip * r."""
    import synthgen as sg
    parts = []
    for k, (ci, co) in enumerate(SHAPES):
        sc = np.sqrt(2.0 / (81 * ci)) * (last_scale if k == 2 else 1.0)
        parts.append(sg.gaussian(seed, k, sc, 81 * co * ci))
    return np.concatenate(parts).astype(np.float32)


def _set_field(lat, U, A, flavour):
    qxd_set_gauge(lat.h, U, A)
    qxd_set_flavour(lat.h, **flavour)
    qxd_clover_build(lat.h)
    qxd_clover_invert(lat.h)


def harvest_and_train(L, cstar, flavour, gauge_seeds, sigma_su3=0.2, sigma_u1=0.3, sources=10, pairs_per_source=10,
                      epochs=8, lr=2e-4, batch=16, skip=None, init_seed=9, source_seed=3500, log=None):
    """Harvest pairs on the fields `gauge_seeds` of an L lattice and train a
    network on them.  Returns (weights, skip, info)."""
    import torch
    import synthgen as sg
    skip = 2.0 * flavour["kappa"] if skip is None else skip
    lat = Lattice(L, cstar)
    Ve = lat.Ve
    vphys = int(np.prod(L))
    fields, spans = [], []
    n_max = len(gauge_seeds) * sources * pairs_per_source
    R = torch.zeros(n_max * 12 * Ve, dtype=torch.complex64, device="cuda")
    E = torch.zeros_like(R)
    t0 = time.perf_counter()
    n = 0
    for f, gs in enumerate(gauge_seeds):
        U = torch.from_numpy(sg.gauge_su3(gs, sigma_su3, vphys)).cuda()
        A = torch.from_numpy(sg.gauge_u1(gs, sigma_u1, vphys)).cuda()
        fields.append((U, A))
        _set_field(lat, U, A, flavour)
        s0 = n
        for src in range(sources):
            b = torch.from_numpy(sg.spinor(source_seed + 100 * f + src, lat.V)).cuda()
            n += qxd_nn_harvest(lat.h, lat.pack(b), pairs_per_source, R[n * 12 * Ve:], E[n * 12 * Ve:])
        spans.append((s0, n))
    torch.cuda.synchronize()
    t_harvest = time.perf_counter() - t0
    net = qxd_nn_create(lat.h)
    qxd_nn_set_weights(net, initial_weights(init_seed))
    qxd_nn_set_skip(net, skip)
    rng = np.random.default_rng(init_seed)
    history = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        tot, cnt = 0.0, 0
        for f in rng.permutation(len(fields)):
            a, b = spans[f]
            if b - a < 1:
                continue
            _set_field(lat, *fields[f], flavour)
            st = qxd_nn_train(lat.h, net, train_params(epochs=1, batch=batch, lr=lr, seed=1000 * ep + int(f), loss=1),
                              R[a * 12 * Ve:b * 12 * Ve], E[a * 12 * Ve:b * 12 * Ve], b - a)
            tot += st["loss_last"] * (b - a)
            cnt += b - a
        history.append(tot / max(cnt, 1))
        if log:
            log("epoch %d: loss %.4f" % (ep + 1, history[-1]))
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    w = qxd_nn_get_weights(net)
    qxd_nn_destroy(net)
    lat.close()
    del R, E
    return w, skip, {"pairs": n, "harvest_s": t_harvest, "train_s": t_train, "loss_history": history}


def make_network(lat, weights, skip):
    """A network on lattice `lat` with the given weights."""
    net = qxd_nn_create(lat.h)
    qxd_nn_set_weights(net, weights)
    qxd_nn_set_skip(net, skip)
    return net
