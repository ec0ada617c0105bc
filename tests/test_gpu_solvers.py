"""GPU solves through the C ABI: FP64 true residual 1e-10 on the full lattice,
checked independently by the oracle, and the solution compared with the
oracle's own CG solution; failure statuses forced from the host."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from tests.gpu_common import make_pair, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

W0 = sg.WORKLOADS["c0"]
FD, FU = sg.FLAVOURS["d"], sg.FLAVOURS["u"]


@pytest.fixture(scope="module")
def c0():
    o, lat, st = make_pair(W0["L"], W0["cstar"], FD, sigma=W0["sigma_su3"], su1=W0["sigma_u1"],
                           seed=W0["gauge_seed"])
    b = sg.spinor(W0["source_seed"], o.V)
    nb = np.linalg.norm(b)
    xe, it, _ = o.cg(o.eo_source(b), 1e-12 * nb)
    x_ref = o.eo_reconstruct(xe, b)
    yield o, lat, b, x_ref
    lat.close()


def _check_solution(o, b, x, x_ref, tag):
    res = np.linalg.norm(b - o.dirac(x)) / np.linalg.norm(b)
    err = np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref)
    print("%s: oracle true residual %.3e, |x - x_oracle|/|x_oracle| %.3e" % (tag, res, err))
    assert res <= 1e-10
    assert err <= 1e-8


def test_cg_f64_c0(c0):
    o, lat, b, x_ref = c0
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F64), x, bd)
    print(st)
    assert st["status"] == 0 and st["true_residual"] <= 1e-10 and st["outer_it"] == 1
    _check_solution(o, b, lat.unpack(x).cpu().numpy(), x_ref, "cg")


@pytest.mark.parametrize("inner", [qxd.F32, qxd.BF16], ids=["f32", "bf16links"])
def test_defect_correction_cg_c0(c0, inner):
    """FP64 defect correction around an FP32 (bf16-link) CG on the normal equations."""
    o, lat, b, x_ref = c0
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=inner), x, bd)
    print(st)
    assert st["status"] == 0 and st["true_residual"] <= 1e-10 and st["outer_it"] >= 2
    _check_solution(o, b, lat.unpack(x).cpu().numpy(), x_ref, "dc-cg%d" % inner)


@pytest.mark.parametrize("inner", [qxd.F64, qxd.F32, qxd.BF16], ids=["f64", "f32", "bf16links"])
def test_fgcr_c0(c0, inner):
    o, lat, b, x_ref = c0
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=inner, nkv=16), None, x, bd)
    print(st)
    assert st["status"] == 0 and st["true_residual"] <= 1e-10
    _check_solution(o, b, lat.unpack(x).cpu().numpy(), x_ref, "fgcr%d" % inner)


def test_solves_are_deterministic(c0):
    o, lat, b, _ = c0
    bd = lat.pack(to_dev(b))
    xs = []
    for _ in range(2):
        x = lat.field(qxd.F64, full=True)
        qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32), None, x, bd)
        xs.append(x)
    assert torch.equal(xs[0], xs[1])


def test_enoconv_when_iteration_limit_hit(c0):
    o, lat, b, _ = c0
    x = lat.field(qxd.F64, full=True)
    for inner in (qxd.F64, qxd.F32):
        st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(nmx=1, res=1e-10, inner_prec=inner), x, lat.pack(to_dev(b)),
                              check=False)
        assert st["status"] == 6
    st = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(nmx=1, res=1e-10), None, x, lat.pack(to_dev(b)), check=False)
    assert st["status"] == 6


def test_enan_on_nan_source(c0):
    o, lat, b, _ = c0
    bb = b.copy()
    bb[3, 1, 2] = np.nan
    x = lat.field(qxd.F64, full=True)
    for inner in (qxd.F64, qxd.F32):
        st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(inner_prec=inner), x, lat.pack(to_dev(bb)), check=False)
        assert st["status"] == 5
    st = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(), None, x, lat.pack(to_dev(bb)), check=False)
    assert st["status"] == 5


def test_esingular_on_exactly_singular_clover():
    """U = 1 and one U(1) link at pi/2: the SW term at x0 + nu is -(u1csw qhat / 8) sigma_{0 nu};
    with u1csw = 32, qhat = 1, kappa = 1/8 one eigenvalue of the block is exactly zero."""
    L = (4, 4, 4, 4)
    lat = qxd.Lattice(L, 0)
    Vp = 4 ** 4
    U = np.broadcast_to(np.eye(3, dtype=complex), (4, Vp, 3, 3)).copy()
    A = np.zeros((4, Vp))
    A[0, 0] = np.pi / 2
    qxd.qxd_set_gauge(lat.h, U, A)
    qxd.qxd_set_flavour(lat.h, qhat=1, invqel=1.0, kappa=0.125, su3csw=0.0, u1csw=32.0)
    qxd.qxd_clover_build(lat.h)
    st = qxd.qxd_clover_invert(lat.h, check=False)
    assert st["status"] == 4 and st["n_singular"] >= 1
    lat.close()


def test_trim_keeps_the_operator_and_blocks_rebuilding():
    """qxd_trim frees the gauge copy and the workspaces: D_hat and solves are
    unchanged afterwards, flavour/clover rebuilds need the gauge field again."""
    o, lat, _ = make_pair((4, 4, 4, 8), 3, FD, sigma=0.2, su1=0.3, seed=5)
    b = sg.spinor(77, o.V)
    bd = lat.pack(to_dev(b))
    psi = lat.pack(to_dev(sg.spinor(78, o.V)))[:12 * lat.Ve].clone()
    before = lat.field(qxd.F64)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, before, psi)
    x0 = lat.field(qxd.F64, full=True)
    qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F64), x0, bd)
    qxd.qxd_trim(lat.h)
    after = lat.field(qxd.F64)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, after, psi)
    assert torch.equal(before, after)
    x1 = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F64), x1, bd)
    assert st["status"] == 0 and torch.equal(x0, x1)
    f = qxd.qxd_flavour(FD["qhat"], FD["invqel"], FD["kappa"], FD["su3csw"], FD["u1csw"])
    assert qxd.load().qxd_set_flavour(lat.h, qxd.ctypes.byref(f), None) == 8
    assert qxd.load().qxd_clover_build(lat.h, None) == 8
    U = sg.gauge_su3(5, 0.2, o.Vphys)
    A = sg.gauge_u1(5, 0.3, o.Vphys)
    lat.setup(U, A, FD)
    again = lat.field(qxd.F64)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, again, psi)
    assert torch.equal(before, again)
    lat.close()


def test_zero_source_gives_the_zero_solution():
    """The degenerate source b = 0: every solver returns x = 0 exactly, status
    OK, no iteration and residual 0, whatever x held before (CG and FGCR in
    every precision and with every preconditioner, the multi-shift solver and
    the rational operator)."""
    L, cstar = (8, 8, 8, 8), 3
    o, lat, _ = make_pair(L, cstar, FD, sigma=0.2, su1=0.3, seed=23)
    zero = lat.field(qxd.F64, full=True)
    net = qxd.qxd_nn_create(lat.h)
    qxd.qxd_nn_set_weights(net, np.full(qxd.NN_NWEIGHTS, 0.01, np.float32))
    d = qxd.qxd_dfl_create(lat.h, 4)
    gen = torch.Generator(device="cuda").manual_seed(3)
    qxd.qxd_dfl_generate(lat.h, d, torch.randn(4 * 24 * lat.Ve, dtype=torch.complex64, device="cuda",
                                               generator=gen), 2, 2, 3)
    cases = [("cg f64", lambda x: qxd.qxd_solve_cg(lat.h, qxd.solver_params(inner_prec=qxd.F64), x, zero)),
             ("cg f32", lambda x: qxd.qxd_solve_cg(lat.h, qxd.solver_params(inner_prec=qxd.F32), x, zero)),
             ("cg bf16", lambda x: qxd.qxd_solve_cg(lat.h, qxd.solver_params(inner_prec=qxd.BF16), x, zero)),
             ("fgcr f64", lambda x: qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(inner_prec=qxd.F64), None, x, zero)),
             ("fgcr f32", lambda x: qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(inner_prec=qxd.F32), None, x, zero)),
             ("fgcr nn", lambda x: qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(inner_prec=qxd.F32), net, x, zero)),
             ("fgcr sap", lambda x: qxd.qxd_solve_fgcr(
                 lat.h, qxd.solver_params(inner_prec=qxd.F32, sap_ncy=2, sap_nmr=4), None, x, zero)),
             ("fgcr dfl", lambda x: qxd.qxd_solve_fgcr_dfl(
                 lat.h, qxd.solver_params(inner_prec=qxd.F32, sap_ncy=2, sap_nmr=4, dfl_nc=4), d, x, zero))]
    for tag, solve in cases:
        x = torch.ones(24 * lat.Ve, dtype=torch.complex128, device="cuda")
        st = solve(x)
        assert st["status"] == 0 and st["inner_it"] == 0 and st["true_residual"] == 0.0, (tag, st)
        assert int(torch.count_nonzero(x)) == 0, tag
    ze = lat.field(qxd.F64)
    xs = [torch.ones(12 * lat.Ve, dtype=torch.complex128, device="cuda") for _ in range(3)]
    st = qxd.qxd_solve_mscg(lat.h, qxd.solver_params(), [0.0, 0.01, 0.1], xs, ze)
    assert st["status"] == 0 and st["inner_it"] == 0 and all(int(torch.count_nonzero(x)) == 0 for x in xs)
    out = torch.ones(12 * lat.Ve, dtype=torch.complex128, device="cuda")
    st = qxd.qxd_rational_apply(lat.h, qxd.solver_params(), 0.5, [0.1, 0.3], [0.2, 0.4], out, ze)
    assert st["status"] == 0 and int(torch.count_nonzero(out)) == 0
    qxd.qxd_dfl_destroy(d)
    qxd.qxd_nn_destroy(net)
    lat.close()

