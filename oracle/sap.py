"""Oracle of the Schwarz alternating procedure (SAP) preconditioner (FP64, test
infrastructure: only tests, the smoke check and the benchmark's CPU leg use it).

SAP is the paper's domain-decomposition preconditioner for GCR (Sec. 4.4, the
SAP+GCR solver; block size, cycles and minimal-residual steps are its
parameters).  Written here from its definition, in plain numpy on the oracle's
own D:

* the extended lattice is cut into 4^4 blocks; block coordinates c = x // 4,
  colour = (c0 + c1 + c2 + c3) mod 2 (neighbouring blocks differ in colour);
* the block operator D_B is D restricted to the sites of B with every hop that
  leaves B dropped (Dirichlet boundary).  For a field rho that vanishes outside
  the blocks of one colour, D(rho) restricted to those blocks is the direct sum
  of the D_B rho_B, because blocks of one colour are never neighbours;
* a block solve is n steps of minimal residual from e = 0 on D_B e = r_B:
  v = D_B rho, alpha = (v, rho) / (v, v) (one alpha per block),
  e += alpha rho, rho -= alpha v;
* one cycle: for colour 0, then colour 1: r = eta - D x, block-solve r on every
  block of that colour, x += e.  M_SAP eta is x after ncy cycles from x = 0.
"""
from __future__ import annotations

import numpy as np

BLOCK = 4


def block_index(o):
    """(block id, colour) of every extended site."""
    x = o.coords(np.arange(o.V))
    nb = [o.Le[m] // BLOCK for m in range(4)]
    c = x // BLOCK
    bid = ((c[:, 0] * nb[1] + c[:, 1]) * nb[2] + c[:, 2]) * nb[3] + c[:, 3]
    colour = (c.sum(axis=1) & 1).astype(np.int8)
    return bid, colour


def supported(o) -> bool:
    """Block colouring consistent with the boundary: an even number (at least
    two) of blocks along every direction, and with C* in k >= 2 the x1 shift L1
    must move an even number of blocks."""
    if any(o.Le[m] % (2 * BLOCK) for m in range(4)):
        return False
    return o.cstar < 2 or (o.L[1] // BLOCK) % 2 == 0


def block_minres(o, r, colour_of_site, colour, bid, nmr):
    """e with D_B e ~ r_B on every block B of the given colour (nmr steps)."""
    mask = (colour_of_site == colour)[:, None, None]
    rho = np.where(mask, r, 0.0)
    e = np.zeros_like(r)
    nblk = int(bid.max()) + 1
    for _ in range(nmr):
        v = np.where(mask, o.dirac(rho), 0.0)
        a = np.bincount(bid, weights=np.sum(np.conj(v) * rho, axis=(1, 2)).real, minlength=nblk) + \
            1j * np.bincount(bid, weights=np.sum(np.conj(v) * rho, axis=(1, 2)).imag, minlength=nblk)
        n = np.bincount(bid, weights=np.sum(np.abs(v) ** 2, axis=(1, 2)), minlength=nblk)
        alpha = np.where(n > 0, a / np.where(n > 0, n, 1.0), 0.0)[bid][:, None, None]
        alpha = np.where(mask, alpha, 0.0)
        e = e + alpha * rho
        rho = rho - alpha * v
    return e


def sap(o, eta, ncy, nmr):
    """M_SAP eta (full-lattice spinor (V, 4, 3) complex)."""
    bid, colour = block_index(o)
    x = np.zeros_like(eta)
    for _ in range(ncy):
        for c in (0, 1):
            r = eta - o.dirac(x)
            x = x + block_minres(o, r, colour, c, bid, nmr)
    return x


def sap_even(o, r_e, ncy, nmr):
    """Preconditioner of the Schur system: (M_SAP (r_e, 0))_e, i.e. SAP on the
    full operator with a source on the even sites, read back on the even sites
    (exact block elimination would give D_hat^-1 r_e)."""
    par = o.parity()
    eta = np.where((par == 0)[:, None, None], r_e, 0.0)
    y = sap(o, eta, ncy, nmr)
    return np.where((par == 0)[:, None, None], y, 0.0)
