"""Pins of the SAP oracle: exact block solves (Dirichlet restriction and the
minimal-residual steps, plain and even-odd preconditioned), the vanishing odd
residual of the even-odd block solve, the multiplicative structure of a cycle,
the block checkerboard along the C* neighbour map, convergence for a heavy quark
and homogeneity."""
import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import sap

FD = sg.FLAVOURS["d"]


def lattice(L=(8, 8, 8, 8), cstar=3, kappa=None):
    o = oracle.Oracle(L, cstar)
    o.set_gauge_physical(sg.gauge_su3(21, 0.2, o.Vphys), sg.gauge_u1(21, 0.3, o.Vphys))
    fl = dict(FD)
    if kappa is not None:
        fl["kappa"] = kappa
    o.set_flavour(**fl, blocks=False)
    return o


@pytest.fixture(scope="module")
def o8():
    return lattice()


@pytest.fixture(scope="module")
def blocks8(o8):
    return sap.site_blocks(o8)


def test_blocks_form_a_checkerboard_along_the_neighbour_map(o8):
    assert sap.supported(o8)
    bid, colour = sap.block_index(o8)
    nb, _ = o8.neighbours()
    for mu in range(4):
        for d in range(2):
            other = nb[:, mu, d]
            cross = bid[other] != bid
            assert np.all(colour[other][cross] != colour[cross])
            assert cross.any()
    # an x1 shift of L1 = 4 sites moves one block: with C* in x2 the colouring breaks
    assert not sap.supported(oracle.Oracle((8, 4, 8, 8), 3))
    assert sap.supported(oracle.Oracle((8, 4, 8, 8), 1))


def test_site_blocks_are_the_diagonal_of_D(o8, blocks8):
    H, Hinv = blocks8
    psi = sg.spinor(4, o8.V)
    one = np.zeros_like(psi)
    s = 77
    one[s] = psi[s]
    # D of a field living on one site, read back on that site
    assert np.allclose(o8.dirac(one)[s].reshape(12), H[s] @ psi[s].reshape(12), rtol=0, atol=1e-13)
    assert np.abs(np.einsum("sij,sjk->sik", H, Hinv) - np.eye(12)).max() < 1e-12


@pytest.mark.parametrize("eo", [False, True])
def test_block_solve_is_exact_with_many_steps(o8, blocks8, eo):
    bid, colour = sap.block_index(o8)
    r = sg.spinor(5, o8.V)
    if eo:
        e = sap.block_minres_eo(o8, r, colour, 0, bid, 120, *blocks8)
    else:
        e = sap.block_minres(o8, r, colour, 0, bid, 250)
    m0 = (colour == 0)[:, None, None]
    assert np.abs(e[~m0[:, 0, 0]]).max() == 0
    res = np.where(m0, r - o8.dirac(e), 0.0)
    print("block residual %.2e" % (np.linalg.norm(res) / np.linalg.norm(np.where(m0, r, 0.0))))
    assert np.linalg.norm(res) <= 1e-11 * np.linalg.norm(np.where(m0, r, 0.0))


def test_eo_block_solve_leaves_no_odd_residual_and_improves_with_steps(o8, blocks8):
    bid, colour = sap.block_index(o8)
    par = o8.parity()
    r = sg.spinor(9, o8.V)
    m1 = colour == 1
    prev = np.inf
    for nmr in (1, 2, 4, 8):
        e = sap.block_minres_eo(o8, r, colour, 1, bid, nmr, *blocks8)
        assert np.abs(e[~m1]).max() == 0
        res = r - o8.dirac(e)
        odd = np.linalg.norm(res[m1 & (par == 1)]) / np.linalg.norm(r[m1])
        even = np.linalg.norm(res[m1 & (par == 0)]) / np.linalg.norm(r[m1])
        print("nmr %d: even residual %.3e, odd %.1e" % (nmr, even, odd))
        assert odd < 1e-13
        assert even <= prev * (1 + 1e-12)
        prev = even
    assert prev < 0.2


@pytest.mark.parametrize("eo", [False, True])
def test_a_cycle_of_exact_block_solves_leaves_no_residual_on_the_last_colour(o8, blocks8, eo):
    bid, colour = sap.block_index(o8)
    eta = sg.spinor(6, o8.V)
    x = sap.sap(o8, eta, 1, 120 if eo else 250, eo, blocks8)
    r = eta - o8.dirac(x)
    last = (colour == 1)
    rel1 = np.linalg.norm(r[last]) / np.linalg.norm(eta[last])
    rel0 = np.linalg.norm(r[~last]) / np.linalg.norm(eta[~last])
    print("residual on colour 1 %.2e, colour 0 %.2e" % (rel1, rel0))
    assert rel1 <= 1e-11
    assert rel0 > 1e-3


@pytest.mark.parametrize("eo", [False, True])
def test_sap_converges_for_a_heavy_quark(eo):
    o = lattice(kappa=0.10)
    blocks = sap.site_blocks(o) if eo else None
    eta = sg.spinor(7, o.V)
    prev = 1.0
    for ncy in (1, 2, 4):
        x = sap.sap(o, eta, ncy, 6, eo, blocks)
        rel = np.linalg.norm(eta - o.dirac(x)) / np.linalg.norm(eta)
        print("ncy %d: %.2e" % (ncy, rel))
        assert rel < 0.5 * prev
        prev = rel
    assert prev < 1e-3


@pytest.mark.parametrize("eo", [False, True])
def test_sap_is_homogeneous(o8, blocks8, eo):
    eta = sg.spinor(8, o8.V)
    c = 0.7 - 1.9j
    a = sap.sap(o8, c * eta, 2, 3, eo, blocks8)
    b = c * sap.sap(o8, eta, 2, 3, eo, blocks8)
    assert np.abs(a - b).max() <= 1e-13 * np.abs(b).max()
