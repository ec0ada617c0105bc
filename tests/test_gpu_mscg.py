"""Multi-shift CG and the rational operator on the GPU through the C ABI.

Parity: every shifted solution against the oracle's own CG for that shift, and
R phi against the oracle's factor-by-factor product, with the paper's printed
[Rational 0] approximation (App. C).  FP64 throughout: the solves stop at a
relative residual of 1e-11, so solutions agree to the conditioning times that
(the bar below is 1e-8, measured about 1e-10), and the oracle recomputes every
GPU residual with its own operator.  At the benchmark sizes: R^4 is the
inverse of D_hat^+ D_hat to 4 delta (the norm bound of App. A.1 taken to the
fourth power), a property that holds at any size."""
import numpy as np
import pytest

import synthgen as sg
from oracle import rational as orat
from tests.gpu_common import from_half64, half64, make_pair
from tests.test_oracle_rational import read_table

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

FD = sg.FLAVOURS["d"]


@pytest.fixture(scope="module", params=[((8, 4, 4, 4), 1), ((8, 4, 4, 4), 3), ((6, 6, 4, 8), 2)],
                ids=["cs1", "cs3", "cs2"])
def pair(request):
    L, cstar = request.param
    o, lat, _ = make_pair(L, cstar, FD, sigma=0.2, su1=0.3, seed=51)
    yield o, lat
    lat.close()


def source(o, seed):
    phi = sg.spinor(seed, o.V)
    phi[o.parity() == 1] = 0
    return phi


@pytest.mark.parametrize("shifts", [[0.0], [0.3], [1e-4, 0.0, 2.5, 1e-2], list(np.geomspace(1e-5, 10.0, 24))],
                         ids=["one", "mu", "four", "max"])
def test_mscg_matches_per_shift_cg(pair, shifts):
    o, lat = pair
    phi = source(o, 52)
    xs = [lat.field(qxd.F64) for _ in shifts]
    st = qxd.qxd_solve_mscg(lat.h, qxd.solver_params(res=1e-11, check_every=2), shifts, xs, half64(lat, phi))
    print("%d shifts: %d iterations, worst true residual %.2e" % (len(shifts), st["inner_it"], st["true_residual"]))
    assert st["status"] == 0 and st["true_residual"] <= 1e-11
    # every residual recomputed by the oracle; solutions compared for the
    # smallest, the largest and one middle shift (the oracle's CG is slow)
    order = np.argsort(shifts)
    compare = {int(order[0]), int(order[-1]), int(order[len(order) // 2])}
    for j, (s, x) in enumerate(zip(shifts, xs)):
        got = from_half64(lat, x)
        res = np.linalg.norm(phi - orat.normal_op(o, got, s)) / np.linalg.norm(phi)
        assert res < 1e-10, (s, res)
        assert np.abs(got[o.parity() == 1]).max() == 0
        if j in compare:
            want = orat.shifted_cg(o, phi, s, tol=1e-12)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            print("  s %.3e: rel err %.2e, oracle residual %.2e" % (s, err, res))
            assert err < 1e-8


@pytest.mark.parametrize("k,l", [(0, 9), (2, 5)], ids=["R", "P_3_6"])
def test_rational_operator_matches_the_oracle(pair, k, l):
    o, lat = pair
    t = read_table()
    A = t["A"] if (k, l) == (0, 9) else 1.0
    nu, mu = t["nu"][k:l + 1], t["mu"][k:l + 1]
    phi = source(o, 53)
    out = lat.field(qxd.F64)
    st = qxd.qxd_rational_apply(lat.h, qxd.solver_params(res=1e-12), A, nu, mu, out, half64(lat, phi))
    got = from_half64(lat, out)
    want = orat.rational_apply(o, phi, A, nu, mu, tol=1e-12)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("factors %d..%d: %d iterations, rel err %.2e" % (k, l, st["inner_it"], err))
    assert st["status"] == 0 and err < 1e-9
    # in place
    inp = half64(lat, phi)
    qxd.qxd_rational_apply(lat.h, qxd.solver_params(res=1e-12), A, nu, mu, inp, inp)
    assert torch.equal(inp, out)


def normal(lat, v):
    t, w = lat.field(qxd.F64), lat.field(qxd.F64)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, t, v)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 1, w, t)
    return w


@pytest.mark.parametrize("work,flav", [("c3", "d"), ("c3", "u"), ("c1", "d")])
def test_fourth_power_of_R_inverts_the_normal_operator(work, flav):
    w = sg.WORKLOADS[work]
    t = read_table()
    lat = qxd.Lattice(w["L"], w["cstar"])
    vp = int(np.prod(w["L"]))
    lat.setup(sg.gauge_su3(w["gauge_seed"], w["sigma_su3"], vp), sg.gauge_u1(w["gauge_seed"], w["sigma_u1"], vp),
              sg.FLAVOURS[flav])
    phi = half64(lat, sg.spinor(w["source_seed"] + 7, lat.V))  # its odd sites are not read
    y = phi.clone()
    its = 0
    for _ in range(4):
        st = qxd.qxd_rational_apply(lat.h, qxd.solver_params(res=1e-12, check_every=8), t["A"], t["nu"], t["mu"], y, y)
        its += st["inner_it"]
    dev = torch.linalg.vector_norm(normal(lat, y) - phi).item() / torch.linalg.vector_norm(phi).item()
    print("%s %s: |M R^4 phi - phi| / |phi| = %.3e (4 delta = %.3e), %d iterations" % (
        work, flav, dev, 4 * t["delta"], its))
    assert dev <= 4 * t["delta"] * (1 + 1e-3) + 1e-9
    lat.close()


def test_mscg_rejects_bad_arguments(pair):
    o, lat = pair
    lib = qxd.load()
    prm = qxd.solver_params()
    b = lat.field(qxd.F64)
    xs = [lat.field(qxd.F64) for _ in range(qxd.QXD_MS_MAXSHIFT + 1)]

    def call(shifts, fields):
        n = len(shifts)
        sh = (qxd.ctypes.c_double * max(n, 1))(*shifts)
        ptrs = (qxd.ctypes.c_void_p * max(n, 1))(*[qxd._ptr(x) for x in fields])
        st = qxd.qxd_solver_stats()
        return lib.qxd_solve_mscg(lat.h, qxd.ctypes.byref(prm), n, sh, ptrs, qxd._ptr(b), qxd.ctypes.byref(st), None)

    assert call([], []) == 1
    assert call([0.1] * (qxd.QXD_MS_MAXSHIFT + 1), xs) == 1
    assert call([-0.1], xs[:1]) == 1
    assert call([float("nan")], xs[:1]) == 1
    assert call([0.1, 0.2], [xs[0], xs[0]]) == 1
    assert call([0.1], [b]) == 1
    out = lat.field(qxd.F64)
    st = qxd.qxd_rational_apply(lat.h, prm, 1.0, [1.0, 2.0], [0.5, 0.5], out, b, check=False)
    assert st["status"] == 1
