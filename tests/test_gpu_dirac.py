"""GPU parity of the operator entry points against the FP64 oracle.

Bars: FP64 1e-13 relative (max-abs error over max-abs value), FP32 1e-6 relative
in norm, BF16 storage reported and loosely gated; pack/unpack bit-exact."""
import numpy as np
import pytest

import synthgen as sg
from tests.gpu_common import even_only, make_pair, norm_err, rel_err, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

FD, FU = sg.FLAVOURS["d"], sg.FLAVOURS["u"]

# several tiles, ragged tails (Ve not a multiple of 256), every cstar, both time signs
GEOMS = [
    ((8, 4, 4, 4), 1, False),      # the 8 x 8 x 4 x 4 extended lattice of the small solve workload
    ((6, 4, 6, 2), 0, False),
    ((4, 6, 2, 6), 2, True),
    ((6, 2, 6, 4), 3, False),
    ((4, 4, 4, 6), 3, True),
    ((2, 2, 2, 2), 3, False),
    ((8, 8, 8, 16), 3, False),     # 8192 even sites: 32 workgroups, windows of the XCD-aware walk
    ((8, 8, 8, 16), 2, True),
]


@pytest.fixture(scope="module", params=GEOMS, ids=lambda g: "L%s_cs%d_t%d" % ("x".join(map(str, g[0])), g[1], g[2]))
def pair(request):
    L, cstar, tanti = request.param
    o, lat, st = make_pair(L, cstar, FD, sigma=0.3, su1=0.4, seed=17, tanti=tanti)
    yield o, lat, st
    lat.close()


def test_pack_unpack_roundtrip_is_exact(pair):
    o, lat, _ = pair
    psi = sg.spinor(5, o.V)
    d = to_dev(psi)
    for prec in (qxd.F64,):
        back = lat.unpack(lat.pack(d, prec), prec).cpu().numpy()
        assert np.array_equal(back, psi)
    # FP32 round trip equals rounding to complex64
    back = lat.unpack(lat.pack(d, qxd.F32), qxd.F32).cpu().numpy()
    assert np.array_equal(back, psi.astype(np.complex64).astype(np.complex128))


def test_dw_apply_f64(pair):
    o, lat, _ = pair
    psi = sg.spinor(11, o.V)
    out = lat.field(qxd.F64, full=True)
    qxd.qxd_dw_apply(lat.h, qxd.F64, out, lat.pack(to_dev(psi)))
    got = lat.unpack(out).cpu().numpy()
    err = rel_err(got, o.dirac(psi))
    assert err < 1e-13


@pytest.mark.parametrize("L,cstar", [((4, 4, 2, 6), 3), ((6, 2, 4, 4), 2)])
def test_up_flavour_dw_and_schur_f64(L, cstar):
    o, lat, _ = make_pair(L, cstar, FU, sigma=0.3, su1=0.4, seed=23)
    psi = sg.spinor(21, o.V)
    out = lat.field(qxd.F64, full=True)
    qxd.qxd_dw_apply(lat.h, qxd.F64, out, lat.pack(to_dev(psi)))
    err = rel_err(lat.unpack(out).cpu().numpy(), o.dirac(psi))
    assert err < 1e-13
    pe = even_only(o, psi)
    x = lat.pack(to_dev(pe))
    out.zero_()
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, out[:12 * lat.Ve], x[:12 * lat.Ve])
    err = rel_err(lat.unpack(out).cpu().numpy(), o.schur(pe))
    assert err < 1e-13
    lat.close()


@pytest.mark.parametrize("dagger", [False, True])
def test_schur_f64(pair, dagger):
    o, lat, _ = pair
    psi = even_only(o, sg.spinor(12, o.V))
    x = lat.pack(to_dev(psi))
    out = lat.field(qxd.F64, full=True)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, dagger, out[:12 * lat.Ve], x[:12 * lat.Ve])
    got = lat.unpack(out).cpu().numpy()
    want = o.schur(psi, dagger=dagger)
    err = rel_err(got, want)
    assert err < 1e-13


@pytest.mark.parametrize("dagger", [False, True])
def test_schur_f32(pair, dagger):
    o, lat, _ = pair
    psi = even_only(o, sg.spinor(13, o.V))
    x = lat.pack(to_dev(psi), qxd.F32)
    out = lat.field(qxd.F32, full=True)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F32, dagger, out[:12 * lat.Ve], x[:12 * lat.Ve])
    got = lat.unpack(out, qxd.F32).cpu().numpy()
    want = o.schur(psi, dagger=dagger)
    err = norm_err(got, want)
    assert err < 1e-6
    err = rel_err(got, want)
    assert err < 5e-6


def test_schur_bf16_storage_error_is_bounded(pair):
    o, lat, _ = pair
    psi = even_only(o, sg.spinor(14, o.V))
    x = lat.pack(to_dev(psi), qxd.BF16)
    out = lat.field(qxd.BF16, full=True)
    qxd.qxd_dw_eo_schur(lat.h, qxd.BF16, False, out[:24 * lat.Ve], x[:24 * lat.Ve])
    got = lat.unpack(out, qxd.BF16).cpu().numpy()
    want = o.schur(psi)
    err = norm_err(got, want)
    print("bf16 storage relative error %.3e" % err)
    assert err < 2e-2


def test_dw_apply_f32(pair):
    o, lat, _ = pair
    psi = sg.spinor(15, o.V)
    out = lat.field(qxd.F32, full=True)
    qxd.qxd_dw_apply(lat.h, qxd.F32, out, lat.pack(to_dev(psi), qxd.F32))
    got = lat.unpack(out, qxd.F32).cpu().numpy()
    err = norm_err(got, o.dirac(psi))
    assert err < 1e-6


def test_eo_source_and_reconstruct(pair):
    o, lat, _ = pair
    b = sg.spinor(16, o.V)
    bd = lat.pack(to_dev(b))
    bh = lat.field(qxd.F64, full=True)
    qxd.qxd_eo_source(lat.h, bh[:12 * lat.Ve], bd)
    err = rel_err(lat.unpack(bh).cpu().numpy(), o.eo_source(b))
    assert err < 1e-13
    xe = even_only(o, sg.spinor(18, o.V))
    x = lat.field(qxd.F64, full=True)
    qxd.qxd_eo_reconstruct(lat.h, x, lat.pack(to_dev(xe))[:12 * lat.Ve], bd)
    err = rel_err(lat.unpack(x).cpu().numpy(), o.eo_reconstruct(xe, b))
    assert err < 1e-13


def test_schur_is_deterministic(pair):
    o, lat, _ = pair
    psi = even_only(o, sg.spinor(19, o.V))
    x = lat.pack(to_dev(psi))
    a = lat.field(qxd.F64, full=True)
    b = lat.field(qxd.F64, full=True)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, a[:12 * lat.Ve], x[:12 * lat.Ve])
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, b[:12 * lat.Ve], x[:12 * lat.Ve])
    assert torch.equal(a, b)


def test_invalid_arguments_are_rejected():
    lat = qxd.Lattice((4, 4, 4, 4), 3)
    f = lat.field(qxd.F64)
    with pytest.raises(qxd.QxdError) as e:  # operator before the clover inverse exists
        qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, f, lat.field(qxd.F64))
    assert e.value.code == 8
    with pytest.raises(qxd.QxdError) as e:  # in place
        qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, f, f)
    assert e.value.code == 1
    lat.close()


@pytest.mark.parametrize("slices", [2, 4])
def test_chunked_schur_order_is_bit_identical(slices):
    """D_hat taken chunk by chunk of time slices (the order the library uses
    on lattices whose chunks hold at least 8 slices, forced here through
    QXD_SCHUR_SLICES on 8 x 16 x 8 x 16 extended, 4 tiles a slice) gives the
    same bits as the two-launch order, with and without the dagger, in FP64
    and FP32, and so does a CG solve, whose norms come from the pass-2
    partial sums."""
    import os
    runs = []
    for s in (0, slices):
        old = os.environ.get("QXD_SCHUR_SLICES")
        os.environ["QXD_SCHUR_SLICES"] = str(s)
        try:
            o, lat, _ = make_pair((8, 8, 8, 16), 3, FD, sigma=0.3, su1=0.4, seed=19)
        finally:
            if old is None:
                del os.environ["QXD_SCHUR_SLICES"]
            else:
                os.environ["QXD_SCHUR_SLICES"] = old
        outs = []
        for prec in (qxd.F64, qxd.F32):
            src = lat.pack(to_dev(sg.spinor(23, o.V)), prec)
            inp = src[: src.numel() // 2].clone()
            for dag in (0, 1):
                out = torch.zeros_like(inp)
                qxd.qxd_dw_eo_schur(lat.h, prec, dag, out, inp)
                outs.append(out.cpu())
        b = lat.pack(to_dev(sg.spinor(24, o.V)))
        x = lat.field(qxd.F64, full=True)
        st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F64), x, b)
        outs.append(x.cpu())
        runs.append((outs, st["inner_it"]))
        lat.close()
    (a, ia), (b_, ib) = runs
    assert ia == ib
    for u, v in zip(a, b_):
        assert torch.equal(u, v)
