"""Inexact deflation (DFL+SAP) on the GPU through the C ABI, against the FP64
oracle from the same seeded start vectors: the vectors after SAP inverse
iteration, the block basis, the little operator (as a dense matrix, blocks
matched by their coordinates) and the two-level preconditioner; FP32 on the
GPU, so the bar is 1e-6 relative, about eight FP32 unit roundoffs (measured
1.2e-7 to 1.8e-7 on both geometries); then DFL-preconditioned
FGCR solves to the FP64 true residual 1e-10 checked by the oracle's D, the
subspace-state errors, and a 32x16^3 solve where deflation cuts the FGCR steps."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import dfl as odfl
from oracle import sap as osap
from tests.gpu_common import from_half32, half32, make_pair, to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

NS, NIT, NCY, NMR = 4, 2, 2, 3


@pytest.fixture(scope="module", params=[((8, 8, 8, 8), 3, 0.136), ((8, 4, 8, 8), 1, 0.145)], ids=["cs3", "cs1"])
def setup(request):
    L, cstar, kappa = request.param
    fl = dict(sg.FLAVOURS["d"])
    fl["kappa"] = kappa
    o, lat, _ = make_pair(L, cstar, fl, sigma=0.2, su1=0.3, seed=21)
    v0 = [sg.spinor(200 + k, o.V) for k in range(NS)]
    vs = odfl.subspace_vectors(o, v0, NIT, NCY, NMR)
    sites, basis = odfl.block_basis(o, vs)
    A = odfl.little_operator(o, sites, basis)
    d = qxd.qxd_dfl_create(lat.h, NS)
    v = torch.cat([lat.pack(to_dev(x), qxd.F32) for x in v0])
    qxd.qxd_dfl_generate(lat.h, d, v, NIT, NCY, NMR)
    torch.cuda.synchronize()
    yield o, lat, d, v, vs, sites, basis, A
    qxd.qxd_dfl_destroy(d)
    lat.close()


def gpu_block_of(o, sites):
    """GPU block number (colour-major, x3 fastest within a colour) of each oracle block."""
    nb = [o.Le[m] // 4 for m in range(4)]
    out = []
    for s in sites:
        c = o.coords(np.array([s[0]]))[0] // 4
        colour = int(c.sum()) & 1
        j = ((c[0] * nb[1] + c[1]) * nb[2] + c[2]) * (nb[3] // 2) + c[3] // 2
        out.append(colour * (np.prod(nb) // 2) + int(j))
    return np.array(out)


def test_inverse_iteration_matches_the_oracle(setup):
    o, lat, d, v, vs, *_ = setup
    n = 24 * lat.Ve
    for k in range(NS):
        got = lat.unpack(v[k * n:(k + 1) * n], qxd.F32).cpu().numpy()
        err = np.linalg.norm(got - vs[k]) / np.linalg.norm(vs[k])
        print("vector %d: %.2e" % (k, err))
        assert err < 1e-6


def test_block_basis_matches_the_oracle(setup):
    o, lat, d, v, vs, sites, basis, A = setup
    worst = 0.0
    for k in range(NS):
        out = lat.field(qxd.F32, full=True)
        qxd.qxd_dfl_basis(lat.h, d, k, out)
        w = lat.unpack(out, qxd.F32).cpu().numpy().reshape(o.V, 12)
        for s, Q in zip(sites, basis):
            worst = max(worst, np.linalg.norm(w[s].reshape(-1) - Q[k]))
    print("basis: max |w_gpu - w_oracle| %.2e" % worst)
    assert worst < 1e-6


def test_little_operator_matches_the_oracle(setup):
    o, lat, d, v, vs, sites, basis, A = setup
    Ag, nbr = qxd.qxd_dfl_little_get(d)
    gb = gpu_block_of(o, sites)
    back = {int(g): b for b, g in enumerate(gb)}
    dense = np.zeros_like(A)
    for R in range(Ag.shape[0]):
        r = back[R]
        for n in range(9):
            c = back[int(nbr[R, n])]
            dense[r * NS:(r + 1) * NS, c * NS:(c + 1) * NS] += Ag[R, n].T  # stored [k][l]
    err = np.abs(dense - A).max() / np.abs(A).max()
    print("little operator: %.2e" % err)
    assert err < 1e-6


@pytest.mark.parametrize("nc,eo", [(2, 0), (8, 0), (8, 1)])
def test_preconditioner_matches_the_oracle(setup, nc, eo):
    o, lat, d, v, vs, sites, basis, A = setup
    r = sg.spinor(31, o.V)
    r[o.parity() == 1] = 0
    out = lat.field(qxd.F32)
    qxd.qxd_dfl_apply(lat.h, d, nc, NCY, NMR, eo, out, half32(lat, r))
    got = from_half32(lat, out)
    blocks = osap.site_blocks(o) if eo else None
    want = odfl.precondition_even(o, sites, basis, A, r, nc, NCY, NMR, bool(eo), blocks)
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("nc %d eo %d: %.2e" % (nc, eo, err))
    assert err < 1e-6


def test_preconditioners_map_zero_to_zero(setup):
    """The degenerate input: SAP and the deflated preconditioner of a vanishing
    residual are exactly zero (the coarse GCR meets a zero norm at its first
    step and must not divide by it)."""
    o, lat, d, *_ = setup
    zero = lat.field(qxd.F32)
    for eo in (0, 1):
        out = torch.ones(12 * lat.Ve, dtype=torch.complex64, device="cuda")
        qxd.qxd_dfl_apply(lat.h, d, 8, NCY, NMR, eo, out, zero)
        assert int(torch.count_nonzero(out)) == 0, eo
        out = torch.ones(12 * lat.Ve, dtype=torch.complex64, device="cuda")
        qxd.qxd_sap_apply(lat.h, NCY, NMR, eo, out, zero)
        assert int(torch.count_nonzero(out)) == 0, eo


@pytest.mark.parametrize("inner", [qxd.F32, qxd.BF16], ids=["f32", "bf16links"])
def test_dfl_fgcr_solves_to_1e10(setup, inner):
    o, lat, d, *_ = setup
    b = sg.spinor(62, o.V)
    x = lat.field(qxd.F64, full=True)
    prm = qxd.solver_params(res=1e-10, inner_prec=inner, sap_ncy=2, sap_nmr=4, sap_plain=1, dfl_nc=8)
    st = qxd.qxd_solve_fgcr_dfl(lat.h, prm, d, x, lat.pack(to_dev(b)))
    print("DFL-FGCR: %d steps, %d applications" % (st["inner_it"], st["sap_applies"]))
    assert st["status"] == 0 and st["true_residual"] <= 1e-10 and st["sap_applies"] >= st["inner_it"]
    res = np.linalg.norm(b - o.dirac(lat.unpack(x).cpu().numpy())) / np.linalg.norm(b)
    assert res <= 1e-10


def test_subspace_state_and_argument_errors(setup):
    o, lat, d, *_ = setup
    lib = qxd.load()
    out, inp = lat.field(qxd.F32), lat.field(qxd.F32)
    P = qxd._ptr
    assert lib.qxd_dfl_apply(lat.h, d, 0, 2, 3, 0, P(out), P(inp), None) == 1
    assert lib.qxd_dfl_apply(lat.h, d, qxd.QXD_DFL_MAXNC + 1, 2, 3, 0, P(out), P(inp), None) == 1
    assert lib.qxd_dfl_apply(lat.h, d, 4, 2, 3, 2, P(out), P(inp), None) == 1
    assert lib.qxd_dfl_apply(lat.h, d, 4, 2, 3, 0, P(out), P(out), None) == 1
    dd = qxd.ctypes.c_void_p()
    assert lib.qxd_dfl_create(lat.h, 0, qxd.ctypes.byref(dd)) == 1
    assert lib.qxd_dfl_create(lat.h, qxd.QXD_DFL_MAXNS + 1, qxd.ctypes.byref(dd)) == 1
    # a new flavour: the little operator belongs to the old operator until rebuilt
    fl = dict(sg.FLAVOURS["u"])
    qxd.qxd_set_flavour(lat.h, **fl)
    qxd.qxd_clover_build(lat.h)
    qxd.qxd_clover_invert(lat.h)
    assert lib.qxd_dfl_apply(lat.h, d, 4, 2, 3, 0, P(out), P(inp), None) == 8
    qxd.qxd_dfl_little(lat.h, d)
    assert lib.qxd_dfl_apply(lat.h, d, 4, 2, 3, 0, P(out), P(inp), None) == 0


def test_dfl_belongs_to_its_lattice_and_operator(setup):
    o, lat, d, *_ = setup
    lib = qxd.load()
    P = qxd._ptr
    other = qxd.Lattice((8, 8, 8, 16), 2)
    vp = 8 * 8 * 8 * 16
    other.setup(sg.gauge_su3(2, 0.2, vp), sg.gauge_u1(2, 0.3, vp), sg.FLAVOURS["d"])
    out, inp = other.field(qxd.F32), other.field(qxd.F32)
    assert lib.qxd_dfl_apply(other.h, d, 4, 2, 3, 0, P(out), P(inp), None) == 1
    assert lib.qxd_dfl_little(other.h, d, None) == 1
    other.close()
    twin = qxd.Lattice(lat.L, lat.cstar)
    vp = int(np.prod(lat.L))
    twin.setup(sg.gauge_su3(21, 0.2, vp), sg.gauge_u1(21, 0.3, vp), sg.FLAVOURS["d"])
    out, inp = twin.field(qxd.F32), twin.field(qxd.F32)
    assert lib.qxd_dfl_apply(twin.h, d, 4, 2, 3, 0, P(out), P(inp), None) == 8
    qxd.qxd_dfl_little(twin.h, d)
    assert lib.qxd_dfl_apply(twin.h, d, 4, 2, 3, 0, P(out), P(inp), None) == 0
    assert lib.qxd_dfl_apply(lat.h, d, 4, 2, 3, 0, P(out), P(inp), None) == 8
    qxd.qxd_dfl_little(lat.h, d)
    twin.close()


def test_dfl_rejects_lattices_sap_does_not_fit():
    lat = qxd.Lattice((8, 4, 8, 8), 3)
    U = sg.gauge_su3(1, 0.2, 8 * 4 * 8 * 8)
    A = sg.gauge_u1(1, 0.3, 8 * 4 * 8 * 8)
    lat.setup(U, A, sg.FLAVOURS["d"])
    dd = qxd.ctypes.c_void_p()
    assert qxd.load().qxd_dfl_create(lat.h, 4, qxd.ctypes.byref(dd)) == 2
    lat.close()


def test_deflation_cuts_fgcr_steps_at_32x16x16x16():
    w = sg.WORKLOADS["c3"]
    vp = int(np.prod(w["L"]))
    fl = dict(sg.FLAVOURS["d"])
    fl["kappa"] = 0.1405
    lat = qxd.Lattice(w["L"], w["cstar"])
    lat.setup(sg.gauge_su3(w["gauge_seed"], w["sigma_su3"], vp), sg.gauge_u1(w["gauge_seed"], w["sigma_u1"], vp), fl)
    b = lat.pack(to_dev(sg.spinor(w["source_seed"], lat.V)))
    gen = torch.Generator(device="cuda").manual_seed(7)
    ns = 16
    v = torch.randn(ns * 24 * lat.Ve, dtype=torch.complex64, device="cuda", generator=gen)
    d = qxd.qxd_dfl_create(lat.h, ns)
    qxd.qxd_dfl_generate(lat.h, d, v, 10, 4, 4)
    x = lat.field(qxd.F64, full=True)
    base = dict(res=1e-10, inner_prec=qxd.F32, sap_ncy=2, sap_nmr=4, sap_plain=1)
    st_sap = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(**base), None, x, b)
    x = lat.field(qxd.F64, full=True)
    st_dfl = qxd.qxd_solve_fgcr_dfl(lat.h, qxd.solver_params(dfl_nc=16, **base), d, x, b)
    print("FGCR steps: SAP %d, DFL+SAP %d" % (st_sap["inner_it"], st_dfl["inner_it"]))
    assert st_dfl["status"] == 0 and st_dfl["true_residual"] <= 1e-10
    assert st_dfl["inner_it"] < st_sap["inner_it"]
    qxd.qxd_dfl_destroy(d)
    lat.close()
