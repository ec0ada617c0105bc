"""The written conventions the paper leaves open, typed once more for the tests.

Chiral gamma basis in 2x2 blocks: g0 = [[0,-1],[-1,0]], gk = [[0,-i s_k],[i s_k,0]];
gamma5 = diag(1,1,-1,-1); sigma_{mu nu} = (i/2)[g_mu, g_nu]; charge conjugation
C = g0 g2.  Both the oracle and the GPU path implement these independently; the
tests use this copy to pin the oracle's results to the closed forms.
"""
import numpy as np

PAULI = [np.array([[0, 1], [1, 0]], complex),
         np.array([[0, -1j], [1j, 0]], complex),
         np.array([[1, 0], [0, -1]], complex)]


def gammas():
    z = np.zeros((2, 2), complex)
    one = np.eye(2, dtype=complex)
    g = [np.block([[z, -one], [-one, z]])]
    for s in PAULI:
        g.append(np.block([[z, -1j * s], [1j * s, z]]))
    return g


GAMMA = gammas()
GAMMA5 = np.diag([1, 1, -1, -1]).astype(complex)
SIGMA = [[0.5j * (GAMMA[m] @ GAMMA[n] - GAMMA[n] @ GAMMA[m]) for n in range(4)] for m in range(4)]
CCONJ = GAMMA[0] @ GAMMA[2]


def spin(mat, psi):
    """Apply a 4x4 spin matrix to a (V, 4, 3) field."""
    return np.einsum("st,vtc->vsc", mat, psi)
