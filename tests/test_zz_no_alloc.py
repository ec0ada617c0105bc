"""The no-allocation Schur entry point (qxd_dw_eo_schur_noalloc) through the C
ABI: its workspace is a static device array, so its output must equal the
allocating entry point's (same kernels, same order: bit for bit) on two calls in
a row, the second on a smaller lattice; a lattice whose odd half field does not
fit the array is rejected with QXD_ESCRATCH before any launch."""
import pytest

import synthgen as sg
from tests.gpu_common import make_pair, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

FD = sg.FLAVOURS["d"]


def _apply_both(lat, o, prec, dagger, seed):
    src = lat.pack(to_dev(sg.spinor(seed, o.V)), prec)
    inp = src[: src.numel() // 2].clone()  # the even half of the full field
    a = torch.zeros_like(inp)
    b = torch.full_like(inp, float("nan"))
    qxd.qxd_dw_eo_schur(lat.h, prec, dagger, a, inp)
    qxd.qxd_dw_eo_schur_noalloc(lat.h, prec, dagger, b, inp)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("prec", [qxd.F64, qxd.F32, qxd.BF16], ids=["f64", "f32", "bf16"])
@pytest.mark.parametrize("dagger", [0, 1])
def test_noalloc_schur_equals_the_allocating_call_twice_in_a_row(prec, dagger):
    # first call: 8 x 16 x 8 x 16 extended (8192 even sites, 32 workgroups);
    # second: 6 x 4 x 6 x 4 extended (288 even sites, a ragged tile)
    for L, seed in (((8, 8, 8, 16), 5), ((6, 2, 6, 4), 6)):
        o, lat, _ = make_pair(L, 3, FD, sigma=0.3, su1=0.4, seed=seed)
        a, b = _apply_both(lat, o, prec, dagger, 100 + seed)
        print("L %s prec %d dagger %d: max |diff| %.3e" % (L, prec, dagger, float((a - b).abs().max())))
        assert torch.equal(a, b)
        assert float(a.abs().max()) > 0
        lat.close()


def test_noalloc_schur_rejects_a_lattice_beyond_the_static_workspace():
    """48 x 24^3 physical with C* in three directions (extended 48 x 48 x 24 x
    24, Ve = 663,552): the FP64 odd half field needs 127 MB and is rejected;
    the FP32 one (63.7 MB) fits and matches the allocating call."""
    vphys = 48 * 24 * 24 * 24
    lat = qxd.Lattice((48, 24, 24, 24), 3)
    assert lat.Ve == 663552
    lat.setup(sg.gauge_su3(2, 0.3, vphys), sg.gauge_u1(2, 0.3, vphys), FD)
    src = lat.pack(to_dev(sg.spinor(7, lat.V)), qxd.F64)
    in64 = src[:12 * lat.Ve].clone()
    out64 = lat.field(qxd.F64)
    P = qxd.ctypes.c_void_p
    code = qxd.load().qxd_dw_eo_schur_noalloc(lat.h, qxd.F64, 0, P(out64.data_ptr()), P(in64.data_ptr()), None)
    assert code == 9 and qxd.qxd_status_string(code) == "QXD_ESCRATCH"
    in32 = lat.pack(to_dev(sg.spinor(7, lat.V)), qxd.F32)[:12 * lat.Ve].clone()
    ref = lat.field(qxd.F32)
    got = lat.field(qxd.F32)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F32, 0, ref, in32)
    qxd.qxd_dw_eo_schur_noalloc(lat.h, qxd.F32, 0, got, in32)
    torch.cuda.synchronize()
    assert torch.equal(ref, got) and float(ref.abs().max()) > 0
    lat.close()


def test_noalloc_schur_needs_the_precision_copies_made_by_an_allocating_call():
    """The FP32 / bf16 operator copies are made by the first allocating call of
    that precision; before it (and after qxd_trim released them) the
    no-allocation call reports QXD_ESTATE instead of allocating."""
    o, lat, _ = make_pair((4, 2, 4, 4), 3, FD, sigma=0.3, su1=0.4, seed=8)
    lib = qxd.load()
    P = qxd.ctypes.c_void_p
    for prec in (qxd.F32, qxd.BF16):
        src = lat.pack(to_dev(sg.spinor(9, o.V)), prec)
        inp = src[: src.numel() // 2].clone()
        out = torch.zeros_like(inp)
        assert lib.qxd_dw_eo_schur_noalloc(lat.h, prec, 0, P(out.data_ptr()), P(inp.data_ptr()), None) == 8
        ref = torch.zeros_like(inp)
        qxd.qxd_dw_eo_schur(lat.h, prec, 0, ref, inp)
        qxd.qxd_dw_eo_schur_noalloc(lat.h, prec, 0, out, inp)
        torch.cuda.synchronize()
        assert torch.equal(ref, out)
    qxd.qxd_trim(lat.h)
    assert lib.qxd_dw_eo_schur_noalloc(lat.h, qxd.BF16, 0, P(out.data_ptr()), P(inp.data_ptr()), None) == 8
    lat.close()
