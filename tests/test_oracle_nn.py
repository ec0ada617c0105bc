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


# ---------------------------------------------------------------------------
# bfloat16 storage mode: rounding points pinned against torch's own
# float32 -> bfloat16 conversion (round to nearest even), closed forms with
# centre-tap weights, and the distance to the exact network.

def _torch_bf16(a):
    torch = pytest.importorskip("torch")
    return torch.from_numpy(np.asarray(a, dtype=np.float64)).float().bfloat16().double().numpy()


def test_bf16_round_matches_torch_and_ties_to_even():
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(200000) * 10.0 ** rng.integers(-30, 30, 200000),
                        # exact ties of the low 16 bits, both parities of the kept half
                        (np.arange(1, 5000, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64),
                        -(np.arange(1, 5000, dtype=np.uint32) << 16 | 0x8000).view(np.float32).astype(np.float64),
                        [0.0, -0.0, 1.0, 1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, 3.0e38, -1.0e-39]])
    got = nn.bf16_round(x)
    assert np.array_equal(got, _torch_bf16(x))
    assert nn.bf16_round(np.array([1.0 + 2.0 ** -8]))[0] == 1.0           # tie, even neighbour below
    assert nn.bf16_round(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6  # tie, even neighbour above
    assert np.array_equal(nn.bf16_round(got), got)


def _centre_weights(c):
    """Weights whose only nonzero tap is d = 0: c[0] [I 0]^T, c[1] I, c[2] [I 0]."""
    W = [np.zeros((81, co, ci)) for ci, co in zip(nn.CHANNELS[:-1], nn.CHANNELS[1:])]
    W[0][40, :24, :] = c[0] * np.eye(24)
    W[1][40] = c[1] * np.eye(32)
    W[2][40, :, :24] = c[2] * np.eye(24)
    return W


def test_bf16_forward_closed_form_with_centre_tap_weights():
    """With centre-tap diagonal weights every layer acts site by site, so the
    rounded network is y = c2 R(max(c1 R(max(c0 R(r), 0)), 0), 0) on each real
    channel (R = bfloat16 rounding, torch's).  The c's are bfloat16 numbers
    whose products with bfloat16 values need rounding again, so leaving out or
    moving any of the three roundings changes the result."""
    o = lattice((4, 2, 2, 4), 3)
    c = (1.0 + 2.0 ** -3 + 2.0 ** -6, 1.0 - 2.0 ** -4 - 2.0 ** -7, 0.75 + 2.0 ** -7)
    assert all(nn.bf16_round(np.array([ci]))[0] == ci for ci in c)
    r = sg.spinor(31, o.V)
    r[o.parity() == 1] = 0
    y, _ = nn.forward(o, _centre_weights(c), r, bf16=True)
    h = nn.embed(o, r)
    want_ch = c[2] * _torch_bf16(np.maximum(c[1] * _torch_bf16(np.maximum(c[0] * _torch_bf16(h), 0.0)), 0.0))
    want = nn.unembed(o, want_ch)
    assert np.abs(y - want).max() <= 1e-15 * np.abs(want).max()
    exact, _ = nn.forward(o, _centre_weights(c), r)
    assert np.abs(exact - want).max() > 1e-4 * np.abs(want).max()


def test_bf16_weight_gradients_closed_form_with_centre_tap_weights():
    """Centre-tap diagonal weights, error loss: the centre-tap weight gradients
    are site sums of rounded gradients times rounded activations,
    dW3 = sum_x g3 h2^T, g2 = R(c2 [I 0]^T g3) [h2 > 0], dW2 = sum_x g2 h1^T,
    g1 = R(c1 g2) [h1 > 0], dW1 = sum_x g1 h0^T, with g3 = R(dL/dy)."""
    o = lattice((4, 2, 2, 4), 3)
    c = (1.0 + 2.0 ** -3 + 2.0 ** -6, 1.0 - 2.0 ** -4 - 2.0 ** -7, 0.75 + 2.0 ** -7)
    W = _centre_weights(c)
    par = o.parity()
    r = sg.spinor(32, o.V)
    e = sg.spinor(33, o.V)
    r[par == 1] = 0
    e[par == 1] = 0
    L, grads = nn.loss_and_grad(o, W, [r], [e], kind=0, bf16=True)
    n = np.linalg.norm(r)
    rh, eh = r / n, e / n
    h0 = _torch_bf16(nn.embed(o, rh))
    h1 = _torch_bf16(np.maximum(c[0] * np.pad(h0, ((0, 0), (0, 8))), 0.0))
    h2 = _torch_bf16(np.maximum(c[1] * h1, 0.0))
    y = nn.unembed(o, c[2] * h2[:, :24])
    d = y - eh
    ne2 = np.vdot(eh, eh).real
    assert abs(L - np.vdot(d, d).real / ne2) <= 1e-13 * L
    g3 = _torch_bf16(nn.embed(o, 2.0 * d / ne2))
    g2 = _torch_bf16(c[2] * np.pad(g3, ((0, 0), (0, 8)))) * (h2 > 0)
    g1 = _torch_bf16(c[1] * g2) * (h1 > 0)
    want = [g1.T @ h0, g2.T @ h1, g3.T @ h2]
    for k in range(3):
        assert np.abs(grads[k][40] - want[k]).max() <= 1e-13 * np.abs(want[k]).max(), k


@pytest.mark.parametrize("kind", [0, 1])
def test_bf16_network_stays_within_bf16_bounds_of_the_exact_one(kind):
    """Random weights: the rounded network and its gradients differ from the
    exact ones by bfloat16-sized amounts (rounding on, but no gross change)."""
    o = lattice()
    o.set_gauge_physical(sg.gauge_su3(3, 0.3, o.Vphys), sg.gauge_u1(3, 0.3, o.Vphys))
    o.set_flavour(**sg.FLAVOURS["d"])
    W = weights(11, scale=1.5)
    par = o.parity()
    r = sg.spinor(101, o.V)
    e = sg.spinor(201, o.V)
    r[par == 1] = 0
    e[par == 1] = 0
    y, _ = nn.forward(o, W, r)
    yb, _ = nn.forward(o, W, r, bf16=True)
    dy = np.linalg.norm(yb - y) / np.linalg.norm(y)
    assert 1e-4 < dy < 2e-2, dy
    L, g = nn.loss_and_grad(o, W, [r], [e], kind)
    Lb, gb = nn.loss_and_grad(o, W, [r], [e], kind, bf16=True)
    assert abs(Lb - L) < 2e-2 * L
    for k in range(3):
        dg = np.linalg.norm(gb[k] - g[k]) / np.linalg.norm(g[k])
        assert 1e-4 < dg < 5e-2, (k, dg)
