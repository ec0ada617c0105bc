"""Pins of the deflation oracle (DFL+SAP, Sec. 4.4): the block basis is
orthonormal and spans the restrictions of the subspace vectors; the little
operator couples a block only to itself and its face neighbours and equals
W^+ D W on every coarse vector; an exact coarse correction leaves no coarse
residual; coarse GCR minimises the residual step by step and is exact after as
many steps as the coarse dimension; inverse iteration lowers |D v| / |v|; and a
subspace built that way cuts the GCR steps of a light quark below SAP alone."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import dfl, sap


def lattice(L=(8, 4, 8, 8), cstar=1, kappa=0.145):
    o = oracle.Oracle(L, cstar)
    o.set_gauge_physical(sg.gauge_su3(21, 0.2, o.Vphys), sg.gauge_u1(21, 0.3, o.Vphys))
    fl = dict(sg.FLAVOURS["d"])
    fl["kappa"] = kappa
    o.set_flavour(**fl, blocks=False)
    return o


@pytest.fixture(scope="module")
def small():
    """cstar 3 lattice, 32 blocks, a 4-vector subspace after two SAP rounds."""
    o = lattice((8, 8, 8, 8), 3, 0.136)
    v0 = [sg.spinor(200 + k, o.V) for k in range(4)]
    vs = dfl.subspace_vectors(o, v0, 2, 2, 3)
    sites, basis = dfl.block_basis(o, vs)
    A = dfl.little_operator(o, sites, basis)
    return o, vs, sites, basis, A


def test_block_basis_is_orthonormal_and_spans_the_restrictions(small):
    o, vs, sites, basis, _ = small
    for s, Q in zip(sites, basis):
        assert np.abs(Q.conj() @ Q.T - np.eye(len(Q))).max() < 1e-12
        for v in vs:
            r = v.reshape(o.V, 12)[s].reshape(-1)
            assert np.linalg.norm(r - Q.T @ (Q.conj() @ r)) < 1e-12 * np.linalg.norm(r)


def test_little_operator_couples_face_neighbours_only(small):
    o, _, sites, basis, A = small
    bid, _ = sap.block_index(o)
    nb, _ = o.neighbours()
    nblk, ns = len(basis), basis[0].shape[0]
    for b in range(nblk):
        touching = set(bid[nb[sites[b]].reshape(-1)]) | {b}
        assert 2 <= len(touching) <= 9
        for b2 in range(nblk):
            blk = A[b * ns:(b + 1) * ns, b2 * ns:(b2 + 1) * ns]
            if b2 in touching:
                assert np.abs(blk).max() > 0
            else:
                assert np.abs(blk).max() == 0


def test_little_operator_is_w_dagger_d_w(small):
    o, _, sites, basis, A = small
    c = np.random.default_rng(5).standard_normal((len(basis), 4)) + 1j
    want = dfl.restrict(o, sites, basis, o.dirac(dfl.prolong(o, sites, basis, c))).reshape(-1)
    assert np.linalg.norm(A @ c.reshape(-1) - want) < 1e-12 * np.linalg.norm(want)


def test_exact_coarse_correction_leaves_no_coarse_residual(small):
    o, _, sites, basis, A = small
    eta = sg.spinor(7, o.V)
    b = dfl.restrict(o, sites, basis, eta).reshape(-1)
    psi = dfl.prolong(o, sites, basis, np.linalg.solve(A, b).reshape(len(basis), -1))
    res = dfl.restrict(o, sites, basis, eta - o.dirac(psi))
    assert np.linalg.norm(res) < 1e-12 * np.linalg.norm(b)


def test_coarse_gcr_minimises_step_by_step_and_ends_exact(small):
    _, _, _, basis, A = small
    b = np.random.default_rng(6).standard_normal(A.shape[0]) + 0.5j
    prev = np.linalg.norm(b)
    for nc in (1, 2, 4, 8, 16, 32):
        c = dfl.coarse_gcr(A, b, nc)
        res = np.linalg.norm(b - A @ c)
        assert res <= prev * (1 + 1e-12)
        prev = res
    c = dfl.coarse_gcr(A, b, A.shape[0])
    assert np.linalg.norm(c - np.linalg.solve(A, b)) < 1e-9 * np.linalg.norm(c)


def test_inverse_iteration_lowers_the_rayleigh_quotient(small):
    o = small[0]
    v0 = [sg.spinor(300 + k, o.V) for k in range(2)]
    prev = [np.linalg.norm(o.dirac(v)) / np.linalg.norm(v) for v in v0]
    for nit in (1, 3):
        vs = dfl.subspace_vectors(o, v0, nit, 2, 3)
        now = [np.linalg.norm(o.dirac(v)) for v in vs]
        assert all(a < b for a, b in zip(now, prev))
        prev = now


def test_deflation_cuts_the_gcr_steps_of_a_light_quark():
    o = lattice()
    b = sg.spinor(3, o.V)
    _, it_sap = dfl.gcr(o, b, lambda r: sap.sap(o, r, 2, 4), 1e-8, nmx=300)
    vs = dfl.subspace_vectors(o, [sg.spinor(100 + k, o.V) for k in range(16)], 10, 4, 4)
    sites, basis = dfl.block_basis(o, vs)
    A = dfl.little_operator(o, sites, basis)
    x, it_dfl = dfl.gcr(o, b, lambda r: dfl.precondition(o, sites, basis, A, r, 16, 2, 4), 1e-8, nmx=300)
    print("GCR steps: SAP %d, DFL+SAP %d" % (it_sap, it_dfl))
    assert np.linalg.norm(b - o.dirac(x)) <= 1e-8 * np.linalg.norm(b)
    assert it_dfl < 0.5 * it_sap
