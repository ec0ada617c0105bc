"""Pins of the rational-operator oracle against the paper's printed [Rational 0]
approximation (App. C) and against dense linear algebra on a tiny lattice:
the printed delta is the maximum relative error of rho over the printed range
and the error alternates in sign with that size at the 22 printed points
(App. A.1); the partial fractions of App. A.2 reproduce the product; shifted
CG and the factor-by-factor rational operator agree with a dense solve and with
the spectral definition rho(D_hat^+ D_hat); the norm bound of App. A.1 holds."""
import os

import numpy as np
import pytest

import oracle
import synthgen as sg
from oracle import rational as orat

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rational0.txt")


def read_table(path=GOLDEN):
    t = {}
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        t[key] = [float(v) for v in vals]
    p, q = t["power"]
    return dict(alpha=-p / q, degree=int(t["degree"][0]), ra=t["range"][0], rb=t["range"][1], muhat=t["mu"][0],
                delta=t["delta"][0], A=t["A"][0], nu=np.array(t["nu"]), mu=np.array(t["mus"]), x=np.array(t["x"]))


@pytest.fixture(scope="module")
def table():
    t = read_table()
    assert t["degree"] == len(t["nu"]) == len(t["mu"]) == 10 and len(t["x"]) == 22
    return t


def test_printed_delta_is_the_maximum_relative_error(table):
    t = table
    q2 = np.geomspace(t["ra"] ** 2, t["rb"] ** 2, 400001)
    e = np.abs(orat.rel_error(q2, t["A"], t["nu"], t["mu"], t["alpha"], t["muhat"]))
    print("max error %.10e, printed delta %.10e" % (e.max(), t["delta"]))
    assert e.max() <= t["delta"] * (1 + 1e-6)
    assert e.max() >= t["delta"] * (1 - 1e-4)


def test_error_alternates_at_the_printed_points(table):
    t = table
    # the end points of the printed range are the first and last points
    assert abs(t["x"][0] / t["ra"] ** 2 - 1) < 1e-12 and abs(t["x"][-1] / t["rb"] ** 2 - 1) < 1e-12
    e = orat.rel_error(t["x"], t["A"], t["nu"], t["mu"], t["alpha"], t["muhat"])
    print(np.array2string(e / t["delta"], precision=7))
    assert np.all(np.abs(np.abs(e) / t["delta"] - 1) < 1e-5)
    assert np.all(np.sign(e[1:]) == -np.sign(e[:-1]))


@pytest.mark.parametrize("k,l", [(0, 9), (0, 4), (5, 8), (9, 9)])
def test_partial_fractions_reproduce_the_product(table, k, l):
    nu, mu = table["nu"][k:l + 1], table["mu"][k:l + 1]
    sig = orat.sigma(nu, mu)
    x = np.geomspace(1e-7, 1e3, 57)
    prod = orat.rho(x, 1.0, nu, mu)
    pf = 1.0 + sum(s / (x + m * m) for s, m in zip(sig, mu))
    assert np.abs(pf / prod - 1).max() < 1e-11


@pytest.fixture(scope="module")
def dense():
    """A 4^4 lattice (no C*) and the dense matrix of D_hat^+ D_hat on its even
    sites, with its eigen-decomposition."""
    o = oracle.Oracle((4, 4, 4, 4), 0)
    o.set_gauge_physical(sg.gauge_su3(31, 0.2, o.Vphys), sg.gauge_u1(31, 0.3, o.Vphys))
    fl = dict(sg.FLAVOURS["d"])
    fl["kappa"] = 0.125
    o.set_flavour(**fl)
    even = np.nonzero(o.parity() == 0)[0]
    n = 12 * len(even)
    cols = np.empty((n, n), dtype=np.complex128)
    for i in range(n):
        v = np.zeros((o.V, 4, 3), dtype=np.complex128)
        v.reshape(o.V, 12)[even[i // 12], i % 12] = 1.0
        cols[:, i] = orat.normal_op(o, v).reshape(o.V, 12)[even].reshape(n)
    lam, vec = np.linalg.eigh(0.5 * (cols + cols.conj().T))
    return o, even, cols, lam, vec


def _flat(o, even, v):
    return v.reshape(o.V, 12)[even].reshape(-1)


def _source(o, seed):
    phi = sg.spinor(seed, o.V)
    phi[o.parity() == 1] = 0
    return phi


def test_dense_operator_is_hermitian_positive(dense):
    o, even, M, lam, _ = dense
    assert np.abs(M - M.conj().T).max() < 1e-12 * np.abs(M).max()
    print("spectrum of D_hat^+ D_hat: [%.4e, %.4e]" % (lam[0], lam[-1]))
    assert lam[0] > 0


@pytest.mark.parametrize("s", [0.0, 1e-3, 0.3])
def test_shifted_cg_matches_a_dense_solve(dense, s):
    o, even, M, _, _ = dense
    phi = _source(o, 32)
    x = orat.shifted_cg(o, phi, s, tol=1e-13)
    want = np.linalg.solve(M + s * np.eye(len(M)), _flat(o, even, phi))
    err = np.linalg.norm(_flat(o, even, x) - want) / np.linalg.norm(want)
    print("s %g: %.2e" % (s, err))
    assert err < 1e-11
    assert np.abs(x[o.parity() == 1]).max() == 0


def test_rational_operator_is_rho_of_the_normal_operator(dense, table):
    o, even, M, lam, vec = dense
    t = table
    phi = _source(o, 33)
    got = _flat(o, even, orat.rational_apply(o, phi, t["A"], t["nu"], t["mu"], tol=1e-13))
    f = _flat(o, even, phi)
    want = vec @ (orat.rho(lam, t["A"], t["nu"], t["mu"]) * (vec.conj().T @ f))
    err = np.linalg.norm(got - want) / np.linalg.norm(want)
    print("rational operator vs spectral: %.2e" % err)
    assert err < 1e-10


def test_norm_bound_of_the_printed_approximation(dense, table):
    o, even, M, lam, vec = dense
    t = table
    assert t["ra"] ** 2 <= lam[0] and lam[-1] <= t["rb"] ** 2
    f = _flat(o, even, _source(o, 34))
    r = vec @ (lam ** t["alpha"] * orat.rho(lam, t["A"], t["nu"], t["mu"]) * (vec.conj().T @ f))
    bound = np.linalg.norm(f - r) / np.linalg.norm(f)
    print("|1 - M^1/4 R| phi / |phi| = %.3e (delta %.3e)" % (bound, t["delta"]))
    assert bound <= t["delta"]
