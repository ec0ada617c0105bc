"""Pins of the network oracle: tap geometry, adjointness, chain rule by finite
differences, homogeneity and translation equivariance."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import nn


def lattice(L=(2, 2, 2, 4), cstar=3):
    return oracle.Oracle(L, cstar)


def weights(seed, scale=0.3):
    out = []
    for k, (ci, co) in enumerate(zip(nn.CHANNELS[:-1], nn.CHANNELS[1:])):
        out.append(sg.gaussian(seed, k, scale / np.sqrt(81 * ci), 81 * co * ci).reshape(81, co, ci))
    return out


@pytest.mark.parametrize("d", [(1, -1, 0, 1), (0, 0, -1, -1), (-1, 1, 1, 0), (0, 0, 0, 0)])
def test_single_tap_is_a_shift_along_the_neighbour_map(d):
    o = lattice((4, 2, 4, 2), 3)
    nb, _ = o.neighbours()
    tap = 27 * (d[0] + 1) + 9 * (d[1] + 1) + 3 * (d[2] + 1) + (d[3] + 1)
    W = np.zeros((81, 5, 5))
    W[tap] = np.eye(5)
    h = sg.gaussian(3, 0, 1.0, o.V * 5).reshape(o.V, 5)
    tgt = np.arange(o.V)
    for mu in range(4):
        if d[mu] == 1:
            tgt = nb[tgt, mu, 0]
        elif d[mu] == -1:
            tgt = nb[tgt, mu, 1]
    assert np.array_equal(o.nn_conv(W, h), h[tgt])


def test_conv_adjoint_and_weight_gradient():
    o = lattice()
    W = sg.gaussian(1, 0, 1.0, 81 * 7 * 5).reshape(81, 7, 5)
    h = sg.gaussian(2, 0, 1.0, o.V * 5).reshape(o.V, 5)
    g = sg.gaussian(3, 0, 1.0, o.V * 7).reshape(o.V, 7)
    lhs = np.sum(g * o.nn_conv(W, h))
    assert abs(lhs - np.sum(o.nn_conv_adjoint(W, g) * h)) < 1e-12 * abs(lhs)
    dW = sg.gaussian(4, 0, 1.0, W.size).reshape(W.shape)
    assert abs(np.sum(g * o.nn_conv(dW, h)) - np.sum(dW * o.nn_conv_wgrad(g, h, 5, 7))) < 1e-11


@pytest.mark.parametrize("kind", [0, 1])
def test_network_gradients_by_central_differences(kind):
    o = lattice()
    o.set_gauge_physical(sg.gauge_su3(3, 0.3, o.Vphys), sg.gauge_u1(3, 0.3, o.Vphys))
    o.set_flavour(**sg.FLAVOURS["d"])
    W = weights(11, scale=1.5)
    par = o.parity()
    rs, es = [], []
    for k in range(2):
        r = sg.spinor(100 + k, o.V)
        e = sg.spinor(200 + k, o.V)
        r[par == 1] = 0
        e[par == 1] = 0
        rs.append(r)
        es.append(e)
    L0, grads = nn.loss_and_grad(o, W, rs, es, kind)
    rng = np.random.default_rng(0)
    h = 1e-6
    for layer in range(3):
        for _ in range(6):
            idx = tuple(rng.integers(0, n) for n in W[layer].shape)
            Wp = [w.copy() for w in W]
            Wm = [w.copy() for w in W]
            Wp[layer][idx] += h
            Wm[layer][idx] -= h
            fd = (nn.loss_and_grad(o, Wp, rs, es, kind)[0] - nn.loss_and_grad(o, Wm, rs, es, kind)[0]) / (2 * h)
            # central differences: truncation O(h^2), rounding about 1e-16 L0 / h
            tol = 1e-7 * abs(grads[layer][idx]) + 1e-9 * max(1.0, L0)
            assert abs(fd - grads[layer][idx]) <= tol, (layer, idx)


def test_network_is_positively_homogeneous_and_translation_equivariant():
    o = lattice((4, 2, 2, 2), 3)
    W = weights(12, scale=2.0)
    par = o.parity()
    r = sg.spinor(5, o.V)
    r[par == 1] = 0
    y, _ = nn.forward(o, W, r)
    y3, _ = nn.forward(o, W, 3.0 * r)
    assert np.abs(y3 - 3.0 * y).max() < 1e-13 * np.abs(y).max()
    assert np.abs(y[par == 1]).max() == 0
    nb, _ = o.neighbours()
    # translate by two steps in t (keeps parity): (T f)(x) = f(x - 2 e0)
    perm = nb[nb[:, 0, 1], 0, 1]
    yt, _ = nn.forward(o, W, r[perm])
    assert np.abs(yt - y[perm]).max() < 1e-13 * np.abs(y).max()


@pytest.mark.parametrize("L,cstar", [((4, 4, 4, 8), 3), ((8, 4, 4, 4), 1), ((2, 4, 2, 6), 2)])
def test_site_local_forward_equals_the_whole_lattice_forward(L, cstar):
    """The patch evaluation used for sampled outputs at full size reproduces
    the whole-lattice network at every site (patches wider than the lattice
    included: extents 2 and 4 wrap inside the 7^4 patch)."""
    o = lattice(L, cstar)
    W = weights(13, scale=2.0)
    r = sg.spinor(6, o.V)
    r[o.parity() == 1] = 0
    y, _ = nn.forward(o, W, r, skip=0.3)
    sites = np.arange(o.V) if o.V <= 1024 else np.random.default_rng(1).choice(o.V, 300, replace=False)
    ys = nn.forward_sites(o, W, r, sites, skip=0.3)
    assert np.abs(ys - y[sites]).max() <= 1e-13 * np.abs(y).max()
