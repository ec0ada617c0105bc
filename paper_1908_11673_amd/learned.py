"""Training driver of the learned preconditioner (orchestration of C ABI calls).

The network is local and translation invariant, so weights trained on one
lattice apply to any lattice with the same field statistics.  Training pairs
(r, e) belong to a gauge field: the residual-norm loss applies that field's
D_hat, so pairs are harvested and trained field by field (one qxd_nn_train
call per field and pass; the Adam state lives in the network).
"""
from __future__ import annotations

import json
import time

import numpy as np

from . import (Lattice, qxd_clover_build, qxd_clover_invert, qxd_nn_create, qxd_nn_destroy,
               qxd_nn_get_weights, qxd_nn_harvest, qxd_nn_load, qxd_nn_save, qxd_nn_set_skip, qxd_nn_set_weights,
               qxd_nn_train, qxd_set_flavour, qxd_set_gauge, train_params)

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
                      epochs=8, lr=2e-4, batch=16, skip=None, init_seed=9, source_seed=3500, log=None,
                      pairs_per_field=None, max_sources=40):
    """Harvest pairs on the fields `gauge_seeds` of an L lattice and train a
    network on them.  Each field gets `sources` Gaussian sources of up to
    `pairs_per_source` pairs each; with `pairs_per_field` set, sources are
    instead added (at most `max_sources`) until that many pairs are harvested
    on the field.  Returns (weights, skip, info)."""
    import torch
    import synthgen as sg
    skip = 2.0 * flavour["kappa"] if skip is None else skip
    lat = Lattice(L, cstar)
    Ve = lat.Ve
    vphys = int(np.prod(L))
    fields, spans = [], []
    per_field = pairs_per_field if pairs_per_field else sources * pairs_per_source
    n_max = len(gauge_seeds) * per_field
    R = torch.zeros(n_max * 12 * Ve, dtype=torch.complex64, device="cuda")
    E = torch.zeros_like(R)
    t0 = time.perf_counter()
    n = 0
    nsrc_used = []
    for f, gs in enumerate(gauge_seeds):
        U = torch.from_numpy(sg.gauge_su3(gs, sigma_su3, vphys)).cuda()
        A = torch.from_numpy(sg.gauge_u1(gs, sigma_u1, vphys)).cuda()
        fields.append((U, A))
        _set_field(lat, U, A, flavour)
        s0 = n
        src = 0
        while src < (max_sources if pairs_per_field else sources) and n - s0 < per_field:
            want = min(pairs_per_source, per_field - (n - s0))
            b = torch.from_numpy(sg.spinor(source_seed + 100 * f + src, lat.V)).cuda()
            n += qxd_nn_harvest(lat.h, lat.pack(b), want, R[n * 12 * Ve:], E[n * 12 * Ve:])
            src += 1
        nsrc_used.append(src)
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
    return w, skip, {"pairs": n, "harvest_s": t_harvest, "train_s": t_train, "loss_history": history,
                     "pairs_per_field": [b - a for a, b in spans], "sources_per_field": nsrc_used}


def make_network(lat, weights, skip):
    """A network on lattice `lat` with the given weights."""
    net = qxd_nn_create(lat.h)
    qxd_nn_set_weights(net, weights)
    qxd_nn_set_skip(net, skip)
    return net


def save_network(prefix, net, meta):
    """Write the network to `prefix`.qxdnn (qxd_nn_save: weights and skip) and
    the JSON-serialisable `meta` (training seeds, configuration, losses) to
    `prefix`.json."""
    qxd_nn_save(net, prefix + ".qxdnn")
    with open(prefix + ".json", "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)


def load_network(lat, prefix):
    """A network on lattice `lat` read back from `prefix`.qxdnn, and its
    metadata from `prefix`.json."""
    net = qxd_nn_create(lat.h)
    try:
        qxd_nn_load(net, prefix + ".qxdnn")
    except Exception:
        qxd_nn_destroy(net)
        raise
    with open(prefix + ".json") as f:
        meta = json.load(f)
    return net, meta
