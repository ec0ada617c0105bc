"""Full-size parity: the Schur operator on the benchmark lattice (32^3 x 64
physical with C* in three directions, extended 64 x 64 x 32 x 32), in the
launch configuration the benchmark times, checked against the oracle on sampled
even sites, plus the adjoint identity over the whole lattice."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

W = sg.WORKLOADS["c1"]


@pytest.fixture(scope="module", params=["d", "u"])
def big(request):
    flav = sg.FLAVOURS[request.param]
    L = W["L"]
    vphys = L[0] * L[1] * L[2] * L[3]
    U = sg.gauge_su3(W["gauge_seed"], W["sigma_su3"], vphys)
    A = sg.gauge_u1(W["gauge_seed"], W["sigma_u1"], vphys)
    o = oracle.Oracle(L, W["cstar"])
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav, cache=False, blocks=False)
    lat = qxd.Lattice(L, W["cstar"])
    st = lat.setup(U, A, flav)
    print("clover min pivot %.4f" % st["min_pivot"])
    del U, A
    psi = sg.spinor(W["source_seed"], o.V)
    psi[o.parity() == 1] = 0
    yield o, lat, psi
    lat.close()


def _sample(o, n=192, seed=0):
    even = np.nonzero(o.parity() == 0)[0]
    rng = np.random.default_rng(seed)
    s = rng.choice(even, size=n - 8, replace=False)
    # include lattice corners, where every C* boundary crossing happens
    corners = o.site(np.array([[0, 0, 0, 0], [o.Le[0] - 1, o.Le[1] - 1, 0, 0], [0, o.L[1] - 1, o.Le[2] - 1, 1],
                               [1, o.L[1], 0, o.Le[3] - 1], [o.Le[0] - 1, 0, o.Le[2] - 1, o.Le[3] - 1],
                               [0, o.Le[1] - 1, 1, 0], [1, 0, 0, 0], [0, 1, o.Le[2] - 1, o.Le[3] - 2]]))
    corners = corners[o.parity()[corners] == 0]
    return np.concatenate([corners, s])


@pytest.mark.parametrize("dagger", [False, True])
def test_schur_f64_full_size_sampled(big, dagger):
    o, lat, psi = big
    x = lat.pack(to_dev(psi))
    out = lat.field(qxd.F64, full=True)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, dagger, out[:12 * lat.Ve], x[:12 * lat.Ve])
    got = lat.unpack(out).cpu().numpy()
    sites = _sample(o)
    want = o.schur_sites(psi, sites, dagger=dagger)
    err = float(np.abs(got[sites] - want).max() / np.abs(want).max())
    print("full-size FP64 D_hat sampled rel err %.2e over %d sites" % (err, sites.size))
    assert err < 1e-13


def test_schur_f32_full_size_sampled(big):
    o, lat, psi = big
    x = lat.pack(to_dev(psi), qxd.F32)
    out = lat.field(qxd.F32, full=True)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F32, 0, out[:12 * lat.Ve], x[:12 * lat.Ve])
    got = lat.unpack(out, qxd.F32).cpu().numpy()
    sites = _sample(o, seed=1)
    want = o.schur_sites(psi, sites)
    err = float(np.linalg.norm(got[sites] - want) / np.linalg.norm(want))
    print("full-size FP32 D_hat sampled rel err %.2e" % err)
    assert err < 1e-6


def test_schur_adjoint_identity_full_size(big):
    """(phi, D_hat psi) = (D_hat^+ phi, psi) over the whole even lattice, in FP64."""
    o, lat, psi = big
    phi = sg.spinor(W["source_seed"] + 7, o.V)
    phi[o.parity() == 1] = 0
    a = lat.pack(to_dev(psi))[:12 * lat.Ve].clone()
    b = lat.pack(to_dev(phi))[:12 * lat.Ve].clone()
    da, db = lat.field(qxd.F64), lat.field(qxd.F64)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 0, da, a)
    qxd.qxd_dw_eo_schur(lat.h, qxd.F64, 1, db, b)
    lhs = torch.vdot(b, da).item()
    rhs = torch.vdot(db, a).item()
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
