"""Oracle of the RHMC rational operator and of shifted normal solves (FP64).

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
leg use it; the library never does.

What it computes, written from App. A of arXiv:1908.11673 in plain numpy on
the oracle's own Schur operator D_hat (even sites):

* the rational function rho(q^2) = A prod_j (q^2 + nu_j^2) / (q^2 + mu_j^2)
  and its relative error 1 - (q^2 + muhat^2)^alpha rho(q^2) against the
  power it approximates (App. A.1);
* the rational operator R = rho(D_hat^+ D_hat) applied factor by factor: for
  each j a shifted normal solve (D_hat^+ D_hat + mu_j^2)^-1 followed by
  (D_hat^+ D_hat + nu_j^2), then the factor A (App. A.1; the factors commute);
* the partial fractions of a factor P_{k,l} = prod_{j=k..l} (M + nu_j^2) /
  (M + mu_j^2) = 1 + sum_j sigma_j / (M + mu_j^2), with sigma_j as the paper
  gives them (App. A.2);
* shifted normal solves (D_hat^+ D_hat + s) x = phi, each by a conjugate
  gradient of its own: what a multi-shift solver returns for all shifts at
  once (the MSCG solver of the sample input, App. C).
"""
from __future__ import annotations

import numpy as np


def rho(q2, A, nu, mu):
    """A prod_j (q2 + nu_j^2) / (q2 + mu_j^2), elementwise in q2."""
    q2 = np.asarray(q2, dtype=np.float64)
    out = np.full(q2.shape, float(A))
    for n, m in zip(nu, mu):
        out = out * (q2 + n * n) / (q2 + m * m)
    return out


def rel_error(q2, A, nu, mu, alpha, muhat=0.0):
    """1 - (q2 + muhat^2)^alpha rho(q2)."""
    q2 = np.asarray(q2, dtype=np.float64)
    return 1.0 - (q2 + muhat * muhat) ** alpha * rho(q2, A, nu, mu)


def sigma(nu, mu):
    """Partial-fraction coefficients of prod_j (x + nu_j^2) / (x + mu_j^2):
    sigma_j = (nu_j^2 - mu_j^2) prod_{m != j} (nu_m^2 - mu_j^2) / (mu_m^2 - mu_j^2)."""
    nu2 = np.asarray(nu, dtype=np.float64) ** 2
    mu2 = np.asarray(mu, dtype=np.float64) ** 2
    out = np.empty(len(mu2))
    for j in range(len(mu2)):
        s = nu2[j] - mu2[j]
        for m in range(len(mu2)):
            if m != j:
                s *= (nu2[m] - mu2[j]) / (mu2[m] - mu2[j])
        out[j] = s
    return out


def normal_op(o, v, s=0.0):
    """(D_hat^+ D_hat + s) v for an even-site spinor v (odd sites zero)."""
    return o.schur(o.schur(v), dagger=True) + s * v


def shifted_cg(o, phi, s, tol=1e-12, nmx=20000):
    """x with (D_hat^+ D_hat + s) x = phi, |phi - (...) x| <= tol |phi|, by
    plain conjugate gradients from x = 0."""
    x = np.zeros_like(phi)
    r = phi.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    stop = (tol * np.linalg.norm(phi)) ** 2
    for _ in range(nmx):
        if rr <= stop:
            break
        w = normal_op(o, p, s)
        a = rr / np.vdot(p, w).real
        x = x + a * p
        r = r - a * w
        rr_new = np.vdot(r, r).real
        p = r + (rr_new / rr) * p
        rr = rr_new
    else:
        raise RuntimeError("shifted CG did not converge")
    return x


def shifted_solves(o, phi, shifts, tol=1e-12):
    """[(D_hat^+ D_hat + s)^-1 phi for s in shifts], each solved on its own."""
    return [shifted_cg(o, phi, s, tol) for s in shifts]


def rational_apply(o, phi, A, nu, mu, tol=1e-12):
    """A prod_j (D_hat^+ D_hat + nu_j^2) (D_hat^+ D_hat + mu_j^2)^-1 phi."""
    y = phi
    for n, m in zip(nu, mu):
        y = normal_op(o, shifted_cg(o, y, m * m, tol), n * n)
    return A * y
