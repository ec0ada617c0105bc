"""Pins of the FP64 oracle to facts fixed by the paper and by mathematics.

Each test checks the oracle against something other than itself: closed forms
(free-field plane waves with C* momenta, a single excited U(1) link), exact
invariants (gamma5-hermiticity, gauge and translation covariance, antisymmetry
of C T D), brute-force dense linear algebra on tiny lattices, and special cases
(qhat = 0, abelian SU(3) fields).  Each is chosen so that a plausible slip in
the oracle (a dropped term, a wrong sign, a swapped index, a transposed
operand, a missing C* shift) fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import dense
from tests.conventions import CCONJ, GAMMA, GAMMA5, SIGMA, spin

FD = sg.FLAVOURS["d"]
FU = sg.FLAVOURS["u"]

GEOMS = [((4, 2, 2, 2), 0), ((2, 2, 2, 2), 1), ((2, 2, 2, 2), 2), ((2, 2, 2, 2), 3),
         ((4, 2, 4, 2), 3), ((2, 4, 2, 4), 2)]


def make(L, cstar, sigma=0.2, su1=0.3, seed=11, flav=FD, tanti=False, cache=True):
    o = oracle.Oracle(L, cstar, tanti)
    U = sg.gauge_su3(seed, sigma, o.Vphys)
    A = sg.gauge_u1(seed, su1, o.Vphys)
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav, cache=cache)
    return o


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---------------------------------------------------------------- geometry

@pytest.mark.parametrize("L,cstar", GEOMS + [((4, 4, 4, 4), 3), ((6, 4, 2, 4), 2)])
def test_neighbour_map_is_consistent(L, cstar):
    o = oracle.Oracle(L, cstar)
    nb, _ = o.neighbours()
    par = o.parity()
    s = np.arange(o.V)
    for mu in range(4):
        assert np.array_equal(nb[nb[s, mu, 0], mu, 1], s)   # -mu undoes +mu
        assert np.all(par[nb[s, mu, 0]] != par)               # each hop flips parity
    for mu, nu in itertools.combinations(range(4), 2):       # unit steps commute
        assert np.array_equal(nb[nb[s, mu, 0], nu, 0], nb[nb[s, nu, 0], mu, 0])
        assert np.array_equal(nb[nb[s, mu, 0], nu, 1], nb[nb[s, nu, 1], mu, 0])
    assert o.V == L[0] * L[1] * L[2] * L[3] * (2 if cstar else 1)
    assert np.sum(par == 0) == o.V // 2


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        oracle.Oracle((4, 3, 2, 2), 1)
    with pytest.raises(ValueError):
        oracle.Oracle((4, 2, 2, 2), 4)


# ------------------------------------------------------ free-field spectrum

def allowed_momentum(o, n, tanti):
    """C* momenta: p1 = 2 pi n1 / L1ext; for k <= cstar the shifted boundary
    needs exp(i p_k L_k) = exp(i p1 L1), so p_k = pi (2 m_k + n1) / L_k."""
    L, Le = o.L, o.Le
    p = np.zeros(4)
    p[0] = (2 * np.pi * n[0] + (np.pi if tanti else 0.0)) / L[0]
    p[1] = 2 * np.pi * n[1] / Le[1]
    for k in (2, 3):
        if k <= o.cstar:
            p[k] = np.pi * (2 * n[k] + n[1]) / L[k]
        else:
            p[k] = 2 * np.pi * n[k] / L[k]
    return p


def free_field(L, cstar, tanti=False, flav=FD):
    o = oracle.Oracle(L, cstar, tanti)
    U = np.broadcast_to(np.eye(3, dtype=complex), (4, o.Vphys, 3, 3))
    A = np.zeros((4, o.Vphys))
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav)
    return o


@pytest.mark.parametrize("L,cstar", [((4, 4, 2, 2), 0), ((4, 4, 4, 2), 1), ((2, 4, 4, 6), 2),
                                     ((4, 2, 4, 4), 3), ((2, 4, 6, 2), 3)])
@pytest.mark.parametrize("tanti", [False, True])
def test_free_field_plane_waves(L, cstar, tanti):
    o = free_field(L, cstar, tanti)
    x = o.coords(np.arange(o.V))
    rng = np.random.default_rng(5)
    kappa = FD["kappa"]
    for trial in range(6):
        n = [rng.integers(0, o.Le[m]) for m in range(4)]
        p = allowed_momentum(o, n, tanti)
        u = rng.normal(size=4) + 1j * rng.normal(size=4)
        col = rng.normal(size=3) + 1j * rng.normal(size=3)
        phase = np.exp(1j * (x @ p))
        psi = phase[:, None, None] * np.einsum("s,c->sc", u, col)[None]
        M = (1 / (2 * kappa) - np.cos(p).sum()) * np.eye(4) + 1j * sum(np.sin(p[m]) * GAMMA[m] for m in range(4))
        want = phase[:, None, None] * np.einsum("s,c->sc", M @ u, col)[None]
        assert rel(o.dirac(psi), want) < 1e-13


@pytest.mark.parametrize("L,cstar", [((2, 4, 4, 2), 2), ((2, 2, 4, 4), 3)])
def test_free_field_rejects_periodic_momenta_under_cstar(L, cstar):
    """Negative control: with n1 odd, a periodic p_k is not an eigenvector."""
    o = free_field(L, cstar)
    x = o.coords(np.arange(o.V))
    p = np.array([0.0, 2 * np.pi * 1 / o.Le[1], 2 * np.pi / o.L[2], 0.0])
    u = np.array([1, 0.5, 0, 0.2j])
    psi = np.exp(1j * (x @ p))[:, None, None] * np.einsum("s,c->sc", u, np.array([1, 0, 0]))[None]
    M = (1 / (2 * FD["kappa"]) - np.cos(p).sum()) * np.eye(4) + 1j * sum(np.sin(p[m]) * GAMMA[m] for m in range(4))
    want = np.exp(1j * (x @ p))[:, None, None] * np.einsum("s,c->sc", M @ u, np.array([1, 0, 0]))[None]
    assert rel(o.dirac(psi), want) > 1e-3


def test_free_field_eigenvalues_basis_free():
    """Spectrum 1/(2k) - sum cos p +- i sqrt(sum sin^2 p), each 6-fold, over all V momenta."""
    o = free_field((2, 2, 2, 2), 3)
    D = dense.dense_dirac(o)
    ev = np.linalg.eigvals(D)
    want = []
    for n in itertools.product(*[range(o.Le[m]) for m in range(4)]):
        p = allowed_momentum(o, n, False)
        re = 1 / (2 * FD["kappa"]) - np.cos(p).sum()
        im = np.sqrt((np.sin(p) ** 2).sum())
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    want = np.array(want)

    def order(z):
        return z[np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))]
    assert np.abs(order(ev) - order(want)).max() < 1e-12


# -------------------------------------------------------- exact invariants

@pytest.mark.parametrize("L,cstar", GEOMS)
@pytest.mark.parametrize("flav", [FD, FU])
def test_gamma5_hermiticity(L, cstar, flav):
    o = make(L, cstar, flav=flav)
    psi = sg.spinor(1, o.V)
    phi = sg.spinor(2, o.V)
    a = np.vdot(phi, spin(GAMMA5, o.dirac(psi)))
    b = np.vdot(psi, spin(GAMMA5, o.dirac(phi)))
    assert abs(a - np.conj(b)) < 1e-14 * abs(a)


def extended_from_physical(o, f_phys, mirror):
    """Extend a physical-lattice site field to the extended lattice."""
    x = o.coords(np.arange(o.V))
    m = x[:, 1] >= o.L[1]
    x1 = np.where(m, x[:, 1] - o.L[1], x[:, 1])
    sp = x[:, 3] + o.L[3] * (x[:, 2] + o.L[2] * (x1 + o.L[1] * x[:, 0]))
    f = f_phys[sp].copy()
    f[m] = mirror(f[m])
    return f


@pytest.mark.parametrize("L,cstar", GEOMS)
def test_gauge_covariance(L, cstar):
    o = make(L, cstar, seed=21)
    U, A = o.gauge_extended()
    om = extended_from_physical(o, sg.transform_su3(5, 1.0, o.Vphys), np.conj)
    al = extended_from_physical(o, sg.angles(6, 1.0, o.Vphys), np.negative)
    nb, _ = o.neighbours()
    U2 = np.empty_like(U)
    A2 = np.empty_like(A)
    for mu in range(4):
        xp = nb[:, mu, 0]
        U2[mu] = om @ U[mu] @ np.conj(np.swapaxes(om[xp], 1, 2))
        A2[mu] = A[mu] + al - al[xp]
    psi = sg.spinor(3, o.V)
    g = om * np.exp(1j * FD["qhat"] * al)[:, None, None]
    out = o.dirac(psi)
    o2 = oracle.Oracle(L, cstar)
    o2.set_gauge_extended(U2, A2)
    o2.set_flavour(**FD)
    out2 = o2.dirac(np.einsum("vab,vsb->vsa", g, psi))
    assert rel(out2, np.einsum("vab,vsb->vsa", g, out)) < 1e-13


@pytest.mark.parametrize("L,cstar", GEOMS)
def test_translation_covariance(L, cstar):
    o = make(L, cstar, seed=31)
    U, A = o.gauge_extended()
    nb, _ = o.neighbours()
    psi = sg.spinor(4, o.V)
    out = o.dirac(psi)
    for k in range(4):
        perm = nb[:, k, 1]           # (T f)(x) = f(x - e_k)
        o2 = oracle.Oracle(L, cstar)
        o2.set_gauge_extended(U[:, perm], A[:, perm])
        o2.set_flavour(**FD)
        assert rel(o2.dirac(psi[perm]), out[perm]) < 1e-14


@pytest.mark.parametrize("L,cstar", [((2, 2, 2, 2), 1), ((4, 2, 2, 2), 3)])
def test_mirror_translation_is_charge_conjugation(L, cstar):
    """Translating by L1 e1 swaps the physical and mirror halves: same as U -> U*, A -> -A."""
    o = make(L, cstar, seed=41)
    U, A = o.gauge_extended()
    x = o.coords(np.arange(o.V))
    xs = x.copy()
    xs[:, 1] = (xs[:, 1] + o.L[1]) % o.Le[1]
    perm = o.site(xs)
    assert rel(U[:, perm], np.conj(U)) < 1e-15 and rel(A[:, perm], -A) < 1e-15
    o2 = oracle.Oracle(L, cstar)
    o2.set_gauge_extended(np.conj(U), -A)
    o2.set_flavour(**FD)
    psi = sg.spinor(4, o.V)
    assert rel(o2.dirac(psi[perm]), o.dirac(psi)[perm]) < 1e-14


@pytest.mark.parametrize("L,cstar", [((2, 2, 2, 2), 1), ((2, 2, 2, 2), 2), ((2, 2, 2, 2), 3), ((4, 2, 2, 2), 3)])
@pytest.mark.parametrize("flav", [FD, FU])
def test_CTD_antisymmetric(L, cstar, flav):
    """pf(CTD) exists: C T D is antisymmetric (T: translation by L1 e1, C = g0 g2)."""
    o = make(L, cstar, sigma=0.5, su1=0.7, seed=51, flav=flav)
    D = dense.dense_dirac(o)
    x = o.coords(np.arange(o.V))
    xs = x.copy()
    xs[:, 1] = (xs[:, 1] + o.L[1]) % o.Le[1]
    perm = o.site(xs)                      # (T psi)(x) = psi(x + L1 e1)
    n = 12 * o.V
    T = np.zeros((n, n))
    comp = np.arange(n).reshape(o.V, 12)
    T[comp.reshape(-1), comp[perm].reshape(-1)] = 1.0
    C = np.kron(np.eye(o.V), np.kron(CCONJ, np.eye(3)))
    M = C @ T @ D
    assert np.abs(M + M.T).max() < 1e-13 * np.abs(M).max()
    # and the check is not empty: D itself is far from C T-related symmetric forms
    assert np.abs(M - M.T).max() > 0.1


# --------------------------------------------------------- clover closed forms

@pytest.mark.parametrize("cstar", [0, 1, 3])
def test_single_u1_link_clover(cstar):
    """U = 1, A = 0 except A(x0, mu) = theta: the SW term is -qhat c_U1 sin(theta)/8 sigma_{mu nu}
    at x0 + nu and x0 + mu + nu, the opposite at x0 - nu and x0 + mu - nu, zero elsewhere
    (the two plaquettes sharing the link cancel at its ends)."""
    L = (4, 4, 4, 4)
    o = oracle.Oracle(L, cstar)
    theta = 0.37
    U = np.broadcast_to(np.eye(3, dtype=complex), (4, o.Vphys, 3, 3))
    A = np.zeros((4, o.Vphys))
    mu = 2
    xp = np.array([1, 1, 2, 3])
    s_phys = xp[3] + L[3] * (xp[2] + L[2] * (xp[1] + L[1] * xp[0]))
    A[mu, s_phys] = theta
    o.set_gauge_physical(U, A)
    c_u1 = 0.8
    o.set_flavour(qhat=-2, invqel=6.0, kappa=0.13, su3csw=1.7, u1csw=c_u1, cache=False)
    want = {}
    x0 = o.site(xp)
    for nu in range(4):
        if nu == mu:
            continue
        block = (-(-2) * c_u1 * np.sin(theta) / 8.0) * np.kron(SIGMA[mu][nu], np.eye(3))
        up = o.shift(x0, np.eye(4, dtype=int)[nu])
        upm = o.shift(up, np.eye(4, dtype=int)[mu])
        dn = o.shift(x0, -np.eye(4, dtype=int)[nu])
        dnm = o.shift(dn, np.eye(4, dtype=int)[mu])
        for s, sg_ in ((up, 1), (upm, 1), (dn, -1), (dnm, -1)):
            want[s] = want.get(s, 0) + sg_ * block
    if cstar >= 1:  # the mirror link carries -theta
        xm = xp.copy()
        xm[1] += L[1]
        xm0 = o.site(xm)
        for nu in range(4):
            if nu == mu:
                continue
            block = (-(-2) * c_u1 * np.sin(-theta) / 8.0) * np.kron(SIGMA[mu][nu], np.eye(3))
            up = o.shift(xm0, np.eye(4, dtype=int)[nu])
            upm = o.shift(up, np.eye(4, dtype=int)[mu])
            dn = o.shift(xm0, -np.eye(4, dtype=int)[nu])
            dnm = o.shift(dn, np.eye(4, dtype=int)[mu])
            for s, sg_ in ((up, 1), (upm, 1), (dn, -1), (dnm, -1)):
                want[s] = want.get(s, 0) + sg_ * block
    for s in range(o.V):
        got = o.sw_site(s)
        assert np.abs(got - want.get(s, 0)).max() < 1e-15, s
    # the hopping term from x0 to x0 + mu carries exp(i qhat theta)
    blk = np.zeros((12, 12), complex)
    e = np.zeros((o.V, 4, 3), complex)
    xf = o.shift(x0, np.eye(4, dtype=int)[mu])
    for j in range(12):
        e.reshape(o.V, 12)[xf, j] = 1
        blk[:, j] = o.dirac_sites(e, [x0]).reshape(12)
        e.reshape(o.V, 12)[xf, j] = 0
    want_hop = -0.5 * np.kron(np.eye(4) - GAMMA[mu], np.exp(1j * -2 * theta) * np.eye(3))
    assert np.abs(blk - want_hop).max() < 1e-15


def test_abelian_su3_field_tensor_matches_u1_formula():
    """For a diagonal SU(3) field, F_hat from the four leaves equals (i/4) Im of the
    four plaquettes, entry by entry: the paper's U(1) formula with q_el = 1."""
    L = (2, 2, 4, 4)
    o = oracle.Oracle(L, 2)
    th = sg.gauge_u1(61, 0.6, o.Vphys)
    ph = sg.gauge_u1(62, 0.6, o.Vphys)
    U = np.zeros((4, o.Vphys, 3, 3), complex)
    U[..., 0, 0] = np.exp(1j * th)
    U[..., 1, 1] = np.exp(1j * ph)
    U[..., 2, 2] = np.exp(-1j * (th + ph))
    o.set_gauge_physical(U, np.zeros((4, o.Vphys)))
    o.set_flavour(qhat=1, invqel=1.0, kappa=0.13, su3csw=1.0, u1csw=1.0, cache=False)
    ref = {}
    for k, ang in enumerate((th, ph, -(th + ph))):
        r = oracle.Oracle(L, 2)
        r.set_gauge_physical(U * 0 + np.eye(3), ang)
        r.set_flavour(qhat=1, invqel=1.0, kappa=0.13, su3csw=1.0, u1csw=1.0, cache=False)
        ref[k] = r
    for s in range(0, o.V, 7):
        F, _ = o.field_tensors(s)
        for k in range(3):
            _, Ah = ref[k].field_tensors(s)
            assert np.abs(F[:, :, k, k] - Ah).max() < 1e-15
        assert np.abs(F[:, :, 0, 1]).max() < 1e-16


@pytest.mark.parametrize("L,cstar", [((2, 2, 2, 2), 3), ((4, 2, 2, 2), 1)])
def test_clover_is_hermitian_and_field_tensor_antihermitian(L, cstar):
    o = make(L, cstar, sigma=0.6, su1=0.8, seed=71)
    for s in range(o.V):
        F, Ah = o.field_tensors(s)
        assert np.abs(F + np.conj(np.swapaxes(F, 2, 3))).max() < 1e-15
        assert np.abs(F + np.swapaxes(F, 0, 1)).max() < 1e-15
        assert np.abs(Ah.real).max() == 0
        sw = o.sw_site(s)
        assert np.abs(sw - sw.conj().T).max() < 1e-15
        # commutes with gamma5 (block diagonal in chirality)
        g5 = np.kron(GAMMA5, np.eye(3))
        assert np.abs(sw @ g5 - g5 @ sw).max() < 1e-15


# ------------------------------------------------------------ special cases

def test_qhat_zero_ignores_u1_field():
    L, cstar = (2, 2, 2, 4), 3
    o1 = make(L, cstar, flav=dict(FD, qhat=0), su1=0.0)
    o2 = make(L, cstar, flav=dict(FD, qhat=0), su1=0.9)
    psi = sg.spinor(8, o1.V)
    assert rel(o2.dirac(psi), o1.dirac(psi)) < 1e-15


def test_invqel_cancels():
    """q Ahat = qhat (i/4) Im(...) whatever q_el is."""
    L, cstar = (2, 2, 2, 4), 3
    o1 = make(L, cstar, flav=dict(FD, invqel=6.0))
    o2 = make(L, cstar, flav=dict(FD, invqel=3.0))
    psi = sg.spinor(8, o1.V)
    assert rel(o2.dirac(psi), o1.dirac(psi)) < 1e-14


def test_u1_clover_coefficient_scales_linearly():
    """Only the SW term depends on u1csw, linearly, and it is site-diagonal."""
    L, cstar = (2, 2, 2, 4), 2
    a = make(L, cstar, flav=dict(FD, u1csw=0.0))
    b = make(L, cstar, flav=dict(FD, u1csw=1.0))
    c = make(L, cstar, flav=dict(FD, u1csw=2.0))
    psi = sg.spinor(9, a.V)
    da, db, dc = a.dirac(psi), b.dirac(psi), c.dirac(psi)
    assert rel(dc - da, 2 * (db - da)) < 1e-13
    assert np.abs(db - da).max() > 1e-3


# ------------------------------------------------------------ even-odd and solves

@pytest.mark.parametrize("L,cstar", [((2, 2, 2, 2), 0), ((2, 2, 2, 2), 1), ((2, 2, 2, 2), 3), ((4, 2, 2, 2), 2)])
def test_schur_matches_dense_complement(L, cstar):
    o = make(L, cstar, sigma=0.4, su1=0.5, seed=81)
    D = dense.dense_dirac(o)
    ie, io = dense.eo_index(o)
    Dh = dense.dense_schur(D, ie, io)
    psi = sg.spinor(12, o.V)
    par = o.parity()
    psi[par == 1] = 0
    out = o.schur(psi)
    assert np.abs(out[par == 1]).max() == 0
    assert rel(out.reshape(-1)[ie], Dh @ psi.reshape(-1)[ie]) < 1e-13
    outd = o.schur(psi, dagger=True)
    assert rel(outd.reshape(-1)[ie], Dh.conj().T @ psi.reshape(-1)[ie]) < 1e-13
    sites = np.nonzero(par == 0)[0][::3]
    assert rel(o.schur_sites(psi, sites), out[sites]) < 1e-15
    # det D = det D_oo det D_hat
    _, ld = np.linalg.slogdet(D)
    _, ldoo = np.linalg.slogdet(D[np.ix_(io, io)])
    _, ldh = np.linalg.slogdet(Dh)
    assert abs(ld - (ldoo + ldh)) < 1e-10
    s1, _ = np.linalg.slogdet(D)
    s2, _ = np.linalg.slogdet(D[np.ix_(io, io)])
    s3, _ = np.linalg.slogdet(Dh)
    assert abs(s1 - s2 * s3) < 1e-10


@pytest.mark.parametrize("L,cstar", [((2, 2, 2, 2), 3), ((4, 2, 2, 2), 1)])
def test_site_block_is_the_diagonal_of_D(L, cstar):
    o = make(L, cstar, seed=91)
    D = dense.dense_dirac(o)
    for s in range(0, o.V, 5):
        blk = o.site_block(s)
        assert np.abs(blk - D[12 * s:12 * s + 12, 12 * s:12 * s + 12]).max() < 1e-15
        assert np.abs(blk - (o.sw_site(s) + np.eye(12) / (2 * FD["kappa"]))).max() < 1e-14


@pytest.mark.parametrize("L,cstar", [((2, 2, 2, 2), 3), ((4, 2, 2, 4), 1), ((4, 2, 2, 2), 0)])
def test_cg_solution_matches_dense_lu(L, cstar):
    o = make(L, cstar, sigma=0.3, seed=101)
    D = dense.dense_dirac(o)
    b = sg.spinor(13, o.V)
    x_lu = np.linalg.solve(D, b.reshape(-1)).reshape(o.V, 4, 3)
    bh = o.eo_source(b)
    nb = np.linalg.norm(b)
    xe, it, res = o.cg(bh, 1e-12 * nb)
    assert it > 0 and res <= 1e-12 * nb
    x = o.eo_reconstruct(xe, b)
    assert np.linalg.norm(b - o.dirac(x)) / nb < 1e-10
    assert np.linalg.norm(x - x_lu) / np.linalg.norm(x_lu) < 1e-9


def test_cg_on_c0_reaches_true_residual():
    w = sg.WORKLOADS["c0"]
    o = make(w["L"], w["cstar"], sigma=w["sigma_su3"], su1=w["sigma_u1"], seed=w["gauge_seed"])
    b = sg.spinor(w["source_seed"], o.V)
    nb = np.linalg.norm(b)
    xe, it, res = o.cg(o.eo_source(b), 1e-10 * nb)
    x = o.eo_reconstruct(xe, b)
    assert it > 0
    assert np.linalg.norm(b - o.dirac(x)) / nb <= 1e-10


@pytest.mark.parametrize("L,cstar", [((4, 4, 2, 2), 3), ((4, 2, 4, 2), 1), ((2, 4, 2, 4), 2)])
def test_gauge_covariance_through_physical_fields(L, cstar):
    """The gauge rotation the GPU tests apply to physical fields (the mirror
    half then filled from them, as the library does) gives D' g psi = g D psi."""
    from tests.gpu_common import gauge_rotate, rotate_spinor
    o = make(L, cstar, seed=23, flav=FU)
    U = sg.gauge_su3(23, 0.2, o.Vphys)
    A = sg.gauge_u1(23, 0.3, o.Vphys)
    U2, A2, g = gauge_rotate(o, U, A, FU["qhat"], 9)
    o2 = oracle.Oracle(L, cstar)
    o2.set_gauge_physical(U2, A2)
    o2.set_flavour(**FU)
    psi = sg.spinor(4, o.V)
    assert rel(o2.dirac(rotate_spinor(g, psi)), rotate_spinor(g, o.dirac(psi))) < 1e-13


def test_operator_calls_before_the_gauge_field_raise():
    """The C side reads the links and the flavour's tables unchecked: the
    wrapper refuses operator calls until both have been set."""
    o = oracle.Oracle((4, 2, 2, 2), 1)
    psi = np.zeros((o.V, 4, 3), dtype=np.complex128)
    with pytest.raises(RuntimeError):
        o.schur(psi)
    with pytest.raises(RuntimeError):
        o.set_flavour(-2, 1.0 / 6.0, 0.13, 1.0, 0.5)
    U = sg.gauge_su3(1, 0.2, o.Vphys)
    A = sg.gauge_u1(1, 0.3, o.Vphys)
    o.set_gauge_physical(U, A)
    with pytest.raises(RuntimeError):
        o.dirac(psi)
    o.set_flavour(-2, 1.0 / 6.0, 0.13, 1.0, 0.5)
    assert np.all(o.schur(psi) == 0)
