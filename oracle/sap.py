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
* the paper's block solver is the even-odd preconditioned form of these steps
  (Sec. 4.4): with D_B = [[H_ee, D_eo], [D_oe, H_oo]] on the block's even and
  odd sites, the steps run on the Schur complement
  D_hat_B = H_ee - D_eo H_oo^-1 D_oe with source r_e - D_eo H_oo^-1 r_o, and the
  odd half follows as e_o = H_oo^-1 (r_o - D_oe e_e), which leaves no residual
  on the block's odd sites;
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


def site_blocks(o):
    """H(x) = D(x, x), the 12 x 12 clover block with its 1/(2 kappa), on every
    site, and its inverse."""
    H = np.stack([o.site_block(s) for s in range(o.V)])
    return H, np.linalg.inv(H)


def _blockmul(M, v):
    return np.einsum("sij,sj->si", M, v.reshape(-1, 12)).reshape(v.shape)


def block_minres_eo(o, r, colour_of_site, colour, bid, nmr, H, Hinv):
    """e with D_B e ~ r_B on every block B of the given colour: nmr minimal
    residual steps on the block's even-odd Schur complement, then the odd half
    by back substitution.  H, Hinv: site_blocks(o)."""
    par = o.parity()
    m = colour_of_site == colour
    me = (m & (par == 0))[:, None, None]
    mo = (m & (par == 1))[:, None, None]

    def d_oe(v):  # v on the block's even sites -> hops onto its odd sites
        return np.where(mo, o.dirac(v), 0.0)

    def d_eo(v):  # v on the block's odd sites -> hops onto its even sites
        return np.where(me, o.dirac(v), 0.0)

    def dhat(v):
        return np.where(me, _blockmul(H, v), 0.0) - d_eo(np.where(mo, _blockmul(Hinv, d_oe(v)), 0.0))

    r_o = np.where(mo, r, 0.0)
    rho = np.where(me, r, 0.0) - d_eo(np.where(mo, _blockmul(Hinv, r_o), 0.0))
    e = np.zeros_like(r)
    nblk = int(bid.max()) + 1
    for _ in range(nmr):
        v = dhat(rho)
        vr = np.sum(np.conj(v) * rho, axis=(1, 2))
        a = np.bincount(bid, weights=vr.real, minlength=nblk) + 1j * np.bincount(bid, weights=vr.imag, minlength=nblk)
        n = np.bincount(bid, weights=np.sum(np.abs(v) ** 2, axis=(1, 2)), minlength=nblk)
        alpha = np.where(n > 0, a / np.where(n > 0, n, 1.0), 0.0)[bid][:, None, None]
        alpha = np.where(me, alpha, 0.0)
        e = e + alpha * rho
        rho = rho - alpha * v
    e_o = np.where(mo, _blockmul(Hinv, r_o - d_oe(e)), 0.0)
    return e + e_o


def sap(o, eta, ncy, nmr, eo=False, blocks=None):
    """M_SAP eta (full-lattice spinor (V, 4, 3) complex); eo: even-odd
    preconditioned block solves (blocks: site_blocks(o), computed if None)."""
    bid, colour = block_index(o)
    if eo and blocks is None:
        blocks = site_blocks(o)
    x = np.zeros_like(eta)
    for _ in range(ncy):
        for c in (0, 1):
            r = eta - o.dirac(x)
            if eo:
                x = x + block_minres_eo(o, r, colour, c, bid, nmr, *blocks)
            else:
                x = x + block_minres(o, r, colour, c, bid, nmr)
    return x


def sap_even(o, r_e, ncy, nmr, eo=False, blocks=None):
    """Preconditioner of the Schur system: (M_SAP (r_e, 0))_e, i.e. SAP on the
    full operator with a source on the even sites, read back on the even sites
    (exact block elimination would give D_hat^-1 r_e)."""
    par = o.parity()
    eta = np.where((par == 0)[:, None, None], r_e, 0.0)
    y = sap(o, eta, ncy, nmr, eo, blocks)
    return np.where((par == 0)[:, None, None], y, 0.0)
