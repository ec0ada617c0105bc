"""Oracle of the inexactly deflated SAP preconditioner (DFL+SAP), FP64.

Test infrastructure: only the tests, the smoke check and the benchmark's CPU
leg use it; the library never does.

The paper's deflated solver (Sec. 4.4, DFL+SAP+GCR) is inexact deflation: a
deflation subspace built from approximate low modes of D, one subspace per
electric charge, whose block projection is solved only approximately.  Written
here from that description in plain numpy on the oracle's own D, on the same
4^4 blocks as SAP:

* subspace: ns start vectors v_k (inputs); nit rounds of v_k <- M_sap v_k
  (approximate inverse iteration, ncy SAP cycles from zero), each followed by
  v_k <- v_k / |v_k|;
* block basis: on every block B the restrictions of v_0 .. v_{ns-1} are
  orthonormalised in that order (classical Gram-Schmidt):
  w_{B,k} = (v_k|_B - sum_{j<k} (w_{B,j}, v_k|_B) w_{B,j}) / |...|;
  W maps coarse vectors c = (c_{B,k}) to sum_{B,k} c_{B,k} w_{B,k};
* little operator A = W^+ D W: A[(B,l),(B',k)] = (w_{B,l}, D w_{B',k}), non-zero
  only for B' = B or a face neighbour of B;
* coarse solve: nc steps of GCR on A c = W^+ eta from c = 0, no restart
  (classical Gram-Schmidt against the earlier A z_j);
* preconditioner: psi = W c, out = psi + M_sap (eta - D psi).
"""
from __future__ import annotations

import numpy as np

from oracle import sap as osap


def normalise(o, vs):
    return [v / np.linalg.norm(v) for v in vs]


def subspace_vectors(o, v0, nit, ncy, nmr, eo=False, blocks=None):
    """The nit rounds of approximate inverse iteration on the start vectors."""
    vs = [np.array(v, dtype=np.complex128) for v in v0]
    for _ in range(nit):
        vs = normalise(o, [osap.sap(o, v, ncy, nmr, eo, blocks) for v in vs])
    return vs


def block_basis(o, vs):
    """W, per block: the block's site list and its orthonormal basis as an
    (ns, 12 nsite) array (rows w_{B,k}, site-major, 12 components a site)."""
    bid, _ = osap.block_index(o)
    nblk = int(bid.max()) + 1
    sites = [np.nonzero(bid == b)[0] for b in range(nblk)]
    basis = []
    for b in range(nblk):
        R = np.stack([v.reshape(o.V, 12)[sites[b]].reshape(-1) for v in vs])  # (ns, 12 nsite)
        Q = np.zeros_like(R)
        for k in range(len(vs)):
            r = R[k] - sum(np.vdot(Q[j], R[k]) * Q[j] for j in range(k))
            Q[k] = r / np.linalg.norm(r)
        basis.append(Q)
    return sites, basis


def restrict(o, sites, basis, eta):
    """W^+ eta as an (nblk, ns) array."""
    e = eta.reshape(o.V, 12)
    return np.stack([Q.conj() @ e[s].reshape(-1) for s, Q in zip(sites, basis)])


def prolong(o, sites, basis, c):
    """W c as a full-lattice spinor."""
    out = np.zeros((o.V, 12), dtype=np.complex128)
    for s, Q, cb in zip(sites, basis, c):
        out[s] = (cb @ Q).reshape(len(s), 12)
    return out.reshape(o.V, 4, 3)


def little_operator(o, sites, basis):
    """Dense A = W^+ D W, (nblk ns) x (nblk ns)."""
    nblk, ns = len(basis), basis[0].shape[0]
    A = np.zeros((nblk * ns, nblk * ns), dtype=np.complex128)
    for b in range(nblk):
        for k in range(ns):
            c = np.zeros((nblk, ns), dtype=np.complex128)
            c[b, k] = 1.0
            A[:, b * ns + k] = restrict(o, sites, basis, o.dirac(prolong(o, sites, basis, c))).reshape(-1)
    return A


def coarse_gcr(A, b, nc):
    """nc GCR steps on A c = b from c = 0 (no restart)."""
    c = np.zeros_like(b)
    r = b.copy()
    zs, ws = [], []
    for _ in range(nc):
        z = r.copy()
        w = A @ z
        beta = [np.vdot(wj, w) for wj in ws]
        for bj, wj, zj in zip(beta, ws, zs):
            w = w - bj * wj
            z = z - bj * zj
        n = np.linalg.norm(w)
        if n == 0.0:
            break
        w, z = w / n, z / n
        a = np.vdot(w, r)
        c = c + a * z
        r = r - a * w
        zs.append(z)
        ws.append(w)
    return c


def precondition(o, sites, basis, A, eta, nc, ncy, nmr, eo=False, blocks=None):
    """psi + M_sap (eta - D psi) with psi = W c, c from nc coarse GCR steps."""
    b = restrict(o, sites, basis, eta).reshape(-1)
    c = coarse_gcr(A, b, nc).reshape(len(basis), -1)
    psi = prolong(o, sites, basis, c)
    return psi + osap.sap(o, eta - o.dirac(psi), ncy, nmr, eo, blocks)


def precondition_even(o, sites, basis, A, r_e, nc, ncy, nmr, eo=False, blocks=None):
    """Preconditioner of the Schur system: the even sites of the above for
    eta = (r_e, 0)."""
    par = o.parity()
    eta = np.where((par == 0)[:, None, None], r_e, 0.0)
    y = precondition(o, sites, basis, A, eta, nc, ncy, nmr, eo, blocks)
    return np.where((par == 0)[:, None, None], y, 0.0)


def gcr(o, b, precond, tol, nmx=500):
    """Right-preconditioned GCR on D x = b (no restart), for the pins."""
    x = np.zeros_like(b)
    r = b.copy()
    zs, ws = [], []
    nb = np.linalg.norm(b)
    for it in range(nmx):
        if np.linalg.norm(r) <= tol * nb:
            return x, it
        z = precond(r)
        w = o.dirac(z)
        for wj, zj in zip(ws, zs):
            bj = np.vdot(wj, w)
            w = w - bj * wj
            z = z - bj * zj
        n = np.linalg.norm(w)
        w, z = w / n, z / n
        a = np.vdot(w, r)
        x = x + a * z
        r = r - a * w
        zs.append(z)
        ws.append(w)
    return x, nmx
