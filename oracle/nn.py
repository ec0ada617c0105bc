"""Oracle of the learned preconditioner network (FP64, test infrastructure).

The network is a local map on the extended lattice: three 3^4-tap
convolution layers whose taps follow the C* neighbour map, real channels
24 -> 32 -> 32 -> 24, no biases, ReLU after the first two layers.

* Input: an even-site spinor ``r`` (V, 4, 3) complex, embedded on the whole
  lattice with the odd sites set to zero, as 24 real channels per site:
  channel ``2 c + 0`` = Re, ``2 c + 1`` = Im of component ``c = 3 spin + colour``.
* Output: the 24 channels of the last layer read back as a spinor, kept on the
  even sites only.
* Preconditioner use: ``M(r) = |r| (N(r / |r|) + skip r / |r|)`` (skip 0: the
  plain network; the linear skip has no weights).
* Training loss over a batch, with ``rhat = r / |r|``, ``ehat = e / |r|``:
  kind 0: ``mean_i |N(rhat_i) - ehat_i|^2 / |ehat_i|^2``;
  kind 1: ``mean_i |D_hat (N(rhat_i) - ehat_i)|^2 / |rhat_i|^2``, the same error
  in the D_hat^+ D_hat norm (the gradient at the output is 2 D_hat^+ D_hat (y - ehat)).

Weights ``W[l]`` have shape (81, cout, cin); tap = 27(d0+1)+9(d1+1)+3(d2+1)+(d3+1).
Backward is the chain rule written out layer by layer: the data gradient of
a convolution is its adjoint (the oracle's literal scatter), the weight
gradient is the site sum of (output gradient) x (shifted input).

Storage precision (``bf16=True``).  The network's specification keeps FP32
master weights and bfloat16 activations.  With ``bf16=True`` every quantity
that such an implementation stores between layers is rounded to bfloat16
(binary32 rounded to nearest even, then its upper 16 bits rounded to nearest
even): the weights, the embedded input, the two ReLU outputs, the gradient at
the network output and the two masked data gradients; the arithmetic between
those points stays FP64, and the network output and the weight gradients are
not rounded.  This is the reference for a bfloat16-storage implementation;
``bf16=False`` is the exact network.  This module is test infrastructure.
"""
from __future__ import annotations

import numpy as np

CHANNELS = (24, 32, 32, 24)


def bf16_round(a):
    """Nearest bfloat16 value of each entry, returned as float64.

    bfloat16 keeps the sign, the 8 exponent bits and the top 7 fraction bits
    of binary32.  The value is first rounded to binary32 (numpy's cast, to
    nearest even), then the low 16 bits of its encoding are rounded off to
    nearest, ties to the even upper half.  Finite inputs only."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    low = u & 0xFFFF
    up = u >> 16
    up = up + ((low > 0x8000) | ((low == 0x8000) & ((up & 1) == 1)))
    return (up << 16).astype(np.uint32).view(np.float32).astype(np.float64)


def _r(x, bf16):
    return bf16_round(x) if bf16 else x


def _rw(W, bf16):
    return [bf16_round(w) for w in W] if bf16 else W


def embed(o, r):
    par = o.parity()
    h = np.zeros((o.V, 24), dtype=np.float64)
    rr = r.reshape(o.V, 12)
    h[:, 0::2] = rr.real
    h[:, 1::2] = rr.imag
    h[par == 1] = 0.0
    return h


def unembed(o, y):
    par = o.parity()
    out = (y[:, 0::2] + 1j * y[:, 1::2]).reshape(o.V, 4, 3).copy()
    out[par == 1] = 0.0
    return out


def forward(o, W, r, skip=0.0, bf16=False):
    """N(r) + skip r and the activations needed by the backward pass."""
    W = _rw(W, bf16)
    h0 = _r(embed(o, r), bf16)
    a1 = o.nn_conv(W[0], h0)
    h1 = _r(np.maximum(a1, 0.0), bf16)
    a2 = o.nn_conv(W[1], h1)
    h2 = _r(np.maximum(a2, 0.0), bf16)
    a3 = o.nn_conv(W[2], h2)
    y = unembed(o, a3)
    if skip:
        y = y + skip * r * (o.parity() == 0)[:, None, None]
    return y, (h0, a1, h1, a2, h2, a3)


def apply_precond(o, W, r, skip=0.0, bf16=False):
    """M(r) = |r| (N(r/|r|) + skip r/|r|)."""
    n = np.linalg.norm(r)
    y, _ = forward(o, W, r / n, skip, bf16)
    return n * y


def backward(o, W, acts, gy, bf16=False):
    """Weight gradients given dL/dy (an even-site spinor).  The ReLU masks are
    taken where the stored activations are positive (a2 > 0 exactly when the
    rounded ReLU output h2 is)."""
    W = _rw(W, bf16)
    h0, a1, h1, a2, h2, a3 = acts
    g3 = _r(embed(o, gy), bf16)
    dW3 = o.nn_conv_wgrad(g3, h2, 32, 24)
    g2 = _r(o.nn_conv_adjoint(W[2], g3) * (h2 > 0), bf16)
    dW2 = o.nn_conv_wgrad(g2, h1, 32, 32)
    g1 = _r(o.nn_conv_adjoint(W[1], g2) * (h1 > 0), bf16)
    dW1 = o.nn_conv_wgrad(g1, h0, 24, 32)
    return [dW1, dW2, dW3]


def loss_and_grad(o, W, rs, es, kind=0, skip=0.0, bf16=False):
    """Batch loss and its weight gradients; ``rs``, ``es`` are lists of spinors."""
    B = len(rs)
    L = 0.0
    grads = [np.zeros_like(w) for w in W]
    for r, e in zip(rs, es):
        n = np.linalg.norm(r)
        rh, eh = r / n, e / n
        y, acts = forward(o, W, rh, skip, bf16)
        d = y - eh
        if kind == 0:
            ne2 = np.vdot(eh, eh).real
            L += np.vdot(d, d).real / ne2 / B
            gy = 2.0 * d / ne2 / B
        else:
            v = o.schur(d)
            nr2 = np.vdot(rh, rh).real
            L += np.vdot(v, v).real / nr2 / B
            gy = 2.0 * o.schur(v, dagger=True) / nr2 / B
        for k, g in enumerate(backward(o, W, acts, gy, bf16)):
            grads[k] += g
    return L, grads


def _patch_conv(Wl, h):
    """One layer on a (n+2)^4 patch of sites: the (n)^4 interior outputs,
    out[a] = sum_d W[tap(d)] h[a + 1 + d]."""
    n = h.shape[0] - 2
    out = np.zeros((n, n, n, n, Wl.shape[1]), dtype=np.float64)
    for tap in range(81):
        d = (tap // 27 - 1, (tap // 9) % 3 - 1, (tap // 3) % 3 - 1, tap % 3 - 1)
        sl = h[1 + d[0]:1 + d[0] + n, 1 + d[1]:1 + d[1] + n, 1 + d[2]:1 + d[2] + n, 1 + d[3]:1 + d[3] + n]
        out += sl @ Wl[tap].T
    return out


def forward_sites(o, W, r, sites, skip=0.0, nb=None, bf16=False):
    """N(r) + skip r at the given sites only, as an (n, 4, 3) array.

    The three layers reach three sites in every direction, so each output
    needs only the 7^4 patch of sites at offsets a in [-3, 3]^4 from it, each
    reached by |a_mu| unit steps of the neighbour map per direction.  Within
    the patch, the site at offset a + d is the tap offset d of the site at
    offset a, because unit steps commute (a C* crossing moves x1 by L1 in
    whichever order the steps are taken).  ``nb``: the neighbour table
    ``o.neighbours()[0]``, if the caller already has it.  ``bf16`` rounds as
    ``forward`` does."""
    W = _rw(W, bf16)
    if nb is None:
        nb, _ = o.neighbours()
    par = o.parity()
    rr = np.asarray(r).reshape(o.V, 12)
    offs = np.stack(np.meshgrid(*[np.arange(-3, 4)] * 4, indexing="ij"), axis=-1).reshape(-1, 4)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for i, s in enumerate(np.asarray(sites)):
        if par[s] == 1:
            continue
        P = np.full(len(offs), int(s), dtype=np.int64)
        for mu in range(4):
            for step in range(1, 4):
                fw, bw = offs[:, mu] >= step, offs[:, mu] <= -step
                P[fw] = nb[P[fw], mu, 0]
                P[bw] = nb[P[bw], mu, 1]
        P = P.reshape(7, 7, 7, 7)
        h0 = np.zeros((7, 7, 7, 7, 24), dtype=np.float64)
        h0[..., 0::2] = rr[P].real
        h0[..., 1::2] = rr[P].imag
        h0[par[P] == 1] = 0.0
        h0 = _r(h0, bf16)
        h1 = _r(np.maximum(_patch_conv(W[0], h0), 0.0), bf16)
        h2 = _r(np.maximum(_patch_conv(W[1], h1), 0.0), bf16)
        y = _patch_conv(W[2], h2)[0, 0, 0, 0]
        out[i] = (y[0::2] + 1j * y[1::2]).reshape(4, 3) + skip * rr[s].reshape(4, 3)
    return out
