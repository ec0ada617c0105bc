"""Maximum size: the largest one-GPU share, 64^3 x 128 physical with C* in
three directions (extended 128 x 128 x 64 x 64, 67,108,864 sites; the FP64
operator takes 97 GB of the GPU, the FP32 copies another 48 GB when used), both
flavours.  The Schur operator in the launch configuration the benchmark times
at this size (windows of 16 tiles per XCD), checked against the oracle on
sampled even sites, including the lattice corners where every C* crossing
happens (FP64 to 1e-13, FP32 to 1e-6); and a mixed-precision CG solve and a
SAP-preconditioned mixed-precision FGCR solve, each checked by the oracle's
residual on sampled sites (the up-type flavour needs about 2830 inner CG
iterations here, about 95 s)."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from tests.gpu_common import to_dev

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
qxd = pytest.importorskip("paper_1908_11673_amd")

W = sg.WORKLOADS["c4"]


@pytest.fixture(scope="module", params=["d", "u"])
def biggest(request):
    flav = sg.FLAVOURS[request.param]
    L = W["L"]
    vphys = int(np.prod(L))
    U = sg.gauge_su3(W["gauge_seed"], W["sigma_su3"], vphys)
    A = sg.gauge_u1(W["gauge_seed"], W["sigma_u1"], vphys)
    print("flavour qhat %+d: generating fields" % flav["qhat"], flush=True)
    o = oracle.Oracle(L, W["cstar"])
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav, cache=False, blocks=False)
    lat = qxd.Lattice(L, W["cstar"])
    st = lat.setup(U, A, flav)
    print("clover min pivot %.4f" % st["min_pivot"], flush=True)
    del U, A
    psi = sg.spinor(W["source_seed"], o.V)
    psi[o.parity() == 1] = 0
    yield o, lat, psi
    lat.close()
    torch.cuda.empty_cache()


def _sample(o, n=128, seed=0):
    even = np.nonzero(o.parity() == 0)[0]
    rng = np.random.default_rng(seed)
    s = rng.choice(even, size=n - 8, replace=False)
    corners = o.site(np.array([[0, 0, 0, 0], [o.Le[0] - 1, o.Le[1] - 1, 0, 0], [0, o.L[1] - 1, o.Le[2] - 1, 1],
                               [1, o.L[1], 0, o.Le[3] - 1], [o.Le[0] - 1, 0, o.Le[2] - 1, o.Le[3] - 1],
                               [0, o.Le[1] - 1, 1, 0], [1, 0, 0, 0], [0, 1, o.Le[2] - 1, o.Le[3] - 2]]))
    corners = corners[o.parity()[corners] == 0]
    return np.concatenate([corners, s])


def _apply(lat, psi, prec, dagger, sites):
    """D_hat (psi) on the GPU, returned at the sampled sites only."""
    x = lat.pack(to_dev(psi), prec)
    out = lat.field(prec, full=True)
    qxd.qxd_dw_eo_schur(lat.h, prec, dagger, out[:out.numel() // 2], x[:x.numel() // 2])
    del x
    got = lat.unpack(out, prec)[torch.from_numpy(sites).cuda()].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    return got


@pytest.mark.parametrize("dagger", [False, True])
def test_schur_f64_max_size_sampled(biggest, dagger):
    o, lat, psi = biggest
    sites = _sample(o)
    got = _apply(lat, psi, qxd.F64, int(dagger), sites)
    want = o.schur_sites(psi, sites, dagger=dagger)
    err = float(np.abs(got - want).max() / np.abs(want).max())
    print("max-size FP64 D_hat sampled rel err %.2e over %d sites" % (err, sites.size))
    assert err < 1e-13


def test_schur_f32_max_size_sampled(biggest):
    o, lat, psi = biggest
    sites = _sample(o, seed=1)
    got = _apply(lat, psi, qxd.F32, 0, sites)
    want = o.schur_sites(psi, sites)
    err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
    print("max-size FP32 D_hat sampled rel err %.2e" % err)
    assert err < 1e-6


def _oracle_residual(o, lat, x, b, seed):
    """The oracle's relative residual |b - D x| on sampled even and odd sites
    (including the corners), after qxd_trim made room for the unpacked x."""
    qxd.qxd_trim(lat.h)  # the solver's workspaces, before the unpacked solution takes their room
    torch.cuda.empty_cache()
    odd = np.nonzero(o.parity() == 1)[0]
    sites = np.concatenate([_sample(o, seed=seed), np.random.default_rng(seed + 1).choice(odd, 64, replace=False)])
    xs = lat.unpack(x)
    xh = np.zeros((o.V, 4, 3), dtype=np.complex128)
    need = np.unique(np.concatenate([sites, o.neighbours()[0][sites].reshape(-1)]))
    xh[need] = xs[torch.from_numpy(need).cuda()].cpu().numpy()
    del xs
    torch.cuda.empty_cache()
    res = np.linalg.norm(b[sites] - o.dirac_sites(xh, sites)) / np.linalg.norm(b[sites])
    print("oracle residual on %d sampled sites: %.2e" % (sites.size, res))
    return res


def test_mixed_precision_cg_solves_at_max_size(biggest):
    """Defect-correction CG (FP32 inner, FP64 outer) at the largest share, after
    qxd_trim drops the gauge copy: the FP64 true residual 1e-10, and the
    oracle's residual on sampled even and odd sites (including the corners);
    the iteration limit bounds the run."""
    o, lat, _ = biggest
    qxd.qxd_trim(lat.h)
    torch.cuda.empty_cache()
    b = sg.spinor(W["source_seed"] + 1, o.V)
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    print("solving", flush=True)
    st = qxd.qxd_solve_cg(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32, check_every=8, nmx=6000), x, bd)
    print("max-size defect-correction CG: %d iterations, true residual %.2e" % (st["inner_it"], st["true_residual"]))
    assert st["status"] == 0 and st["true_residual"] <= 1e-10
    del bd
    assert _oracle_residual(o, lat, x, b, 2) <= 1e-9


def test_sap_fgcr_solves_at_max_size(biggest):
    """SAP-preconditioned FGCR (FP32 inner with 2 SAP cycles of 8 plain
    minimal-residual steps, FP64 defect correction) at the largest share: the
    block-order copies fit beside the FP64 operator with restart length 6 (4 if
    6 does not fit); the FP64 true residual 1e-10 and the oracle's residual on
    sampled sites; the step limit bounds the run."""
    o, lat, _ = biggest
    qxd.qxd_trim(lat.h)
    torch.cuda.empty_cache()
    b = sg.spinor(W["source_seed"] + 2, o.V)
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    for nkv in (6, 4):
        prm = qxd.solver_params(res=1e-10, inner_prec=qxd.F32, sap_ncy=2, sap_nmr=8, sap_plain=1, nkv=nkv, nmx=400)
        print("solving with restart length %d" % nkv, flush=True)
        st = qxd.qxd_solve_fgcr(lat.h, prm, None, x, bd, check=False)
        if st["status"] != 3:  # QXD_ENOMEM: try the shorter restart
            break
        qxd.qxd_trim(lat.h)
        torch.cuda.empty_cache()
    print("max-size SAP-FGCR(%d): %d steps, true residual %.2e" % (nkv, st["inner_it"], st["true_residual"]))
    assert st["status"] == 0 and st["true_residual"] <= 1e-10
    del bd
    assert _oracle_residual(o, lat, x, b, 4) <= 1e-9


def test_enomem_leaves_no_hip_error_for_the_next_call(biggest):
    """A solve whose vectors do not fit (FGCR with restart length 24 beside the
    FP64 operator at the largest share: 48 FP32 directions of 3.2 GB) returns
    QXD_ENOMEM, and the next call succeeds: the failed allocation is not
    reported again as a HIP error (QXD_EHIP)."""
    o, lat, psi = biggest
    qxd.qxd_trim(lat.h)
    torch.cuda.empty_cache()
    b = sg.spinor(W["source_seed"] + 3, o.V)
    bd = lat.pack(to_dev(b))
    x = lat.field(qxd.F64, full=True)
    st = qxd.qxd_solve_fgcr(lat.h, qxd.solver_params(res=1e-10, inner_prec=qxd.F32, nkv=24), None, x, bd,
                            check=False)
    print("FGCR(24) at the largest share: status %d" % st["status"])
    assert st["status"] == 3  # QXD_ENOMEM
    del bd, x
    qxd.qxd_trim(lat.h)
    torch.cuda.empty_cache()
    sites = _sample(o, seed=5)
    got = _apply(lat, psi, qxd.F64, 0, sites)  # raises on any status but QXD_OK
    want = o.schur_sites(psi, sites)
    assert float(np.abs(got - want).max() / np.abs(want).max()) < 1e-13
