"""Learned preconditioner on the GPU, through the C ABI.

Forward and weight gradients are compared with the network oracle in its
bfloat16 storage mode, which rounds the weights, the embedded input, the ReLU
outputs and the back-propagated gradients to bfloat16 where the kernels store
them, on the FP32-rounded input the GPU receives.  What remains is FP32
accumulation on the matrix cores against FP64 in the oracle, and the rare
bfloat16 rounding it flips.  Bars, in norm: every layer's weight gradient
1e-2, the network's tolerance for bfloat16 storage (measured at most 1.9e-3,
layer 1); the output 2e-3 (measured at most 1.8e-4); the loss 1e-4 (measured
at most 1.4e-6).  The distance to the exact FP64 network (4e-3 for outputs, up
to 5.7e-2 for gradients) is printed beside it.  Training, the
preconditioned solve and the fallbacks are checked on the FP64 true
residual."""
import os

import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import nn as onn
from tests.gpu_common import make_pair, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

FD = sg.FLAVOURS["d"]
SHAPES = [(24, 32), (32, 32), (32, 24)]


def init_weights(seed, scale=1.0):
    ws = []
    for k, (ci, co) in enumerate(SHAPES):
        ws.append(sg.gaussian(seed, k, scale * np.sqrt(2.0 / (81 * ci)), 81 * co * ci).reshape(81, co, ci))
    return ws


def flat(ws):
    return np.concatenate([w.reshape(-1) for w in ws]).astype(np.float32)


def f32(a):
    """the FP32 rounding the GPU's input fields receive"""
    return np.asarray(a).astype(np.complex64).astype(np.complex128)


def half32(lat, o, psi):
    """even-site spinor -> FP32 even half field on the device"""
    return lat.pack(to_dev(psi), qxd.F32)[:12 * lat.Ve].clone()


def from_half32(lat, o, t):
    full = lat.field(qxd.F32, full=True)
    full[:12 * lat.Ve] = t
    return lat.unpack(full, qxd.F32).cpu().numpy()


# Lattices whose extended extents are multiples of 4 x 4 x 4 x 8 run the
# block-tiled convolution (cs3_blocks: 2 blocks, C* crossings in x2 and x3;
# cs2_blocks: 2 blocks along t, one along x1..x3, so every halo wraps onto the
# block itself); the others, and "gather", run the per-site kernel.
@pytest.fixture(scope="module", params=[((4, 2, 4, 4), 3, False), ((2, 4, 2, 6), 2, False), ((8, 4, 4, 4), 1, False),
                                        ((4, 4, 4, 8), 3, True), ((4, 4, 4, 8), 3, False), ((8, 2, 4, 8), 2, False)],
                ids=["cs3", "cs2_ragged", "c0", "cs3_gather", "cs3_blocks", "cs2_blocks"])
def lat_pair(request):
    L, cstar, gather = request.param
    o, lat, _ = make_pair(L, cstar, FD, sigma=0.2, su1=0.3, seed=31)
    lat.gather = gather
    yield o, lat
    lat.close()


def new_net(lat):
    """A network on `lat`; the per-site gather kernel when the lattice asks for it."""
    old = os.environ.get("QXD_NN_GATHER")
    os.environ["QXD_NN_GATHER"] = "1" if getattr(lat, "gather", False) else "0"
    try:
        return qxd.qxd_nn_create(lat.h)
    finally:
        if old is None:
            del os.environ["QXD_NN_GATHER"]
        else:
            os.environ["QXD_NN_GATHER"] = old


@pytest.mark.parametrize("skip", [0.0, 0.27])
def test_forward_matches_oracle(lat_pair, skip):
    o, lat = lat_pair
    ws = init_weights(5)
    net = new_net(lat)
    qxd.qxd_nn_set_weights(net, flat(ws))
    qxd.qxd_nn_set_skip(net, skip)
    r = sg.spinor(41, o.V)
    r[o.parity() == 1] = 0
    out = lat.field(qxd.F32)
    qxd.qxd_nn_apply(lat.h, net, out, half32(lat, o, r))
    got = from_half32(lat, o, out)
    want = onn.apply_precond(o, ws, f32(r), skip, bf16=True)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    exact = onn.apply_precond(o, ws, r, skip)
    print("nn forward rel err %.2e (exact FP64 network: %.2e)" % (
        err, np.linalg.norm(got - exact) / np.linalg.norm(exact)))
    assert err < 2e-3
    assert np.abs(got[o.parity() == 1]).max() == 0
    # positive homogeneity: M(2 r) = 2 M(r) exactly
    out2 = lat.field(qxd.F32)
    qxd.qxd_nn_apply(lat.h, net, out2, half32(lat, o, 2 * r))
    assert torch.equal(out2, 2 * out)
    qxd.qxd_nn_destroy(net)


@pytest.mark.parametrize("kind,skip", [(0, 0.0), (1, 0.0), (1, 0.27)],
                         ids=["error_loss", "residual_loss", "residual_loss_skip"])
def test_loss_and_gradient_match_oracle(lat_pair, kind, skip):
    o, lat = lat_pair
    ws = init_weights(6, scale=1.5)
    net = new_net(lat)
    qxd.qxd_nn_set_weights(net, flat(ws))
    qxd.qxd_nn_set_skip(net, skip)
    par = o.parity()
    rs, es = [], []
    for k in range(2):
        r = sg.spinor(50 + k, o.V)
        e = sg.spinor(60 + k, o.V)
        r[par == 1] = 0
        e[par == 1] = 0
        rs.append(r)
        es.append(e)
    R = torch.cat([half32(lat, o, r) for r in rs])
    E = torch.cat([half32(lat, o, e) for e in es])
    loss, grad = qxd.qxd_nn_loss_grad(lat.h, net, R, E, 2, kind)
    L0, g0 = onn.loss_and_grad(o, ws, [f32(r) for r in rs], [f32(e) for e in es], kind, skip, bf16=True)
    Lx, gx = onn.loss_and_grad(o, ws, rs, es, kind, skip)
    print("loss gpu %.6f oracle %.6f (exact %.6f)" % (loss, L0, Lx))
    assert abs(loss - L0) / L0 < 1e-4
    off = 0
    for k, (ci, co) in enumerate(SHAPES):
        n = 81 * co * ci
        gk = grad[off:off + n].reshape(81, co, ci)
        off += n
        err = np.linalg.norm(gk - g0[k]) / np.linalg.norm(g0[k])
        print("layer %d grad rel err %.2e (exact FP64 network: %.2e)" % (
            k + 1, err, np.linalg.norm(gk - gx[k]) / np.linalg.norm(gx[k])))
        assert err < 1e-2
    qxd.qxd_nn_destroy(net)


def test_block_and_gather_kernels_agree():
    """The block-tiled and the per-site convolutions compute the same network
    (up to FP32 summation order and the bf16 roundings it can flip)."""
    o, lat, _ = make_pair((4, 4, 4, 8), 3, FD, sigma=0.2, su1=0.3, seed=32)
    ws = flat(init_weights(7))
    r = sg.spinor(43, o.V)
    r[o.parity() == 1] = 0
    outs = []
    for gather in (False, True):
        lat.gather = gather
        net = new_net(lat)
        qxd.qxd_nn_set_weights(net, ws)
        qxd.qxd_nn_set_skip(net, 0.1)
        out = lat.field(qxd.F32)
        qxd.qxd_nn_apply(lat.h, net, out, half32(lat, o, r))
        outs.append(out.cpu().to(torch.complex128))
        qxd.qxd_nn_destroy(net)
    err = float(torch.linalg.norm(outs[0] - outs[1]) / torch.linalg.norm(outs[1]))
    print("block vs gather rel diff %.2e" % err)
    assert err < 5e-3
    lat.close()


def test_zero_weights_fall_back_and_still_converge(lat_pair):
    o, lat = lat_pair
    net = new_net(lat)
    qxd.qxd_nn_set_weights(net, np.zeros(qxd.NN_NWEIGHTS, np.float32))
    b = sg.spinor(70, o.V)
    x = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32), net, x, lat.pack(to_dev(b)))
    assert st["fell_back"] == 1 and st["true_residual"] <= 1e-10
    res = np.linalg.norm(b - o.dirac(lat.unpack(x).cpu().numpy())) / np.linalg.norm(b)
    assert res <= 1e-10
    qxd.qxd_nn_destroy(net)


def test_nan_weights_fall_back_and_still_converge(lat_pair):
    o, lat = lat_pair
    net = new_net(lat)
    w = flat(init_weights(7))
    w[100] = np.nan
    qxd.qxd_nn_set_weights(net, w)
    b = sg.spinor(71, o.V)
    x = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32), net, x, lat.pack(to_dev(b)))
    assert st["fell_back"] == 1 and st["true_residual"] <= 1e-10
    qxd.qxd_nn_destroy(net)


def test_harvest_pairs_satisfy_the_schur_equation(lat_pair):
    o, lat = lat_pair
    b = sg.spinor(72, o.V)
    n = 6
    R = torch.zeros(n * 12 * lat.Ve, dtype=torch.complex64, device="cuda")
    E = torch.zeros_like(R)
    got = qxd.qxd_nn_harvest(lat.h, lat.pack(to_dev(b)), n, R, E)
    assert got >= 2
    nbh = np.linalg.norm(o.eo_source(b))
    for i in range(got):
        r = from_half32(lat, o, R[i * 12 * lat.Ve:(i + 1) * 12 * lat.Ve])
        e = from_half32(lat, o, E[i * 12 * lat.Ve:(i + 1) * 12 * lat.Ve])
        # D_hat e_k = r_k - r_final: pairs are taken while |r_k| > 1e-6 |bhat|, the
        # final residual is below 1e-10 |b|, and both fields are rounded to FP32
        assert np.linalg.norm(r) >= 0.99e-6 * nbh
        err = np.linalg.norm(o.schur(e) - r) / np.linalg.norm(r)
        assert err < 2e-4, (i, err)


def test_training_lowers_the_loss_and_the_solve_stays_exact():
    """Train field by field on pairs harvested from a few small fields; the
    network-preconditioned solve of a held-out field must still reach the FP64
    true residual (whether the network helps at this toy scale is reported)."""
    L, cstar = (8, 4, 4, 4), 3
    flav = FD
    lat = qxd.Lattice(L, cstar)
    Vp = int(np.prod(L))
    fields, pairs = [], []
    npf = 12
    for seed in range(3):
        U = sg.gauge_su3(300 + seed, 0.2, Vp)
        A = sg.gauge_u1(300 + seed, 0.3, Vp)
        lat.setup(U, A, flav)
        rr, ee = [], []
        for src in range(2):
            b = sg.spinor(400 + 10 * seed + src, lat.V)
            R = torch.zeros(npf * 12 * lat.Ve, dtype=torch.complex64, device="cuda")
            E = torch.zeros_like(R)
            got = qxd.qxd_nn_harvest(lat.h, lat.pack(to_dev(b)), npf, R, E)
            rr.append(R[:got * 12 * lat.Ve])
            ee.append(E[:got * 12 * lat.Ve])
        fields.append((U, A))
        pairs.append((torch.cat(rr), torch.cat(ee)))
    net = qxd.qxd_nn_create(lat.h)
    ws = init_weights(9)
    ws[2] *= 0.05  # start near the zero map
    qxd.qxd_nn_set_weights(net, flat(ws))
    qxd.qxd_nn_set_skip(net, 2 * flav["kappa"])
    first = last = None
    for ep in range(10):
        for f in range(3):
            lat.setup(*fields[f], flav)
            R, E = pairs[f]
            n = R.numel() // (12 * lat.Ve)
            st = qxd.qxd_nn_train(lat.h, net, qxd.train_params(epochs=1, batch=8, lr=2e-4, seed=ep, loss=1), R, E, n)
            if first is None:
                first = st["loss_first"]
            last = st["loss_last"]
    print("training loss %.4f -> %.4f" % (first, last))
    assert last < first
    U = sg.gauge_su3(399, 0.2, Vp)
    A = sg.gauge_u1(399, 0.3, Vp)
    lat.setup(U, A, flav)
    o = oracle.Oracle(L, cstar)
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav)
    b = sg.spinor(499, lat.V)
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    plain = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32, nkv=16), None, x, bd)
    x2 = lat.field(qxd.F64, full=True)
    learned = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32, nkv=16), net, x2, bd)
    print("plain FGCR", plain)
    print("NN FGCR", learned)
    assert learned["true_residual"] <= 1e-10
    res = np.linalg.norm(b - o.dirac(lat.unpack(x2).cpu().numpy())) / np.linalg.norm(b)
    assert res <= 1e-10
    qxd.qxd_nn_destroy(net)
    lat.close()
