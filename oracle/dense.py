"""Dense-matrix tools for tiny lattices (test infrastructure).

The dense operator is read off the oracle column by column (D e_j), so these
tools add no arithmetic of their own beyond numpy's LU and determinants.
"""
from __future__ import annotations

import numpy as np


def dense_dirac(o) -> np.ndarray:
    n = 12 * o.V
    D = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((o.V, 4, 3), dtype=np.complex128)
    for j in range(n):
        e.reshape(-1)[j] = 1.0
        D[:, j] = o.dirac(e).reshape(-1)
        e.reshape(-1)[j] = 0.0
    return D


def eo_index(o):
    """Component indices of the even and the odd sites in the flattened field."""
    par = o.parity()
    comp = np.arange(12 * o.V).reshape(o.V, 12)
    return comp[par == 0].reshape(-1), comp[par == 1].reshape(-1)


def dense_schur(D, ie, io):
    Dee = D[np.ix_(ie, ie)]
    Deo = D[np.ix_(ie, io)]
    Doe = D[np.ix_(io, ie)]
    Doo = D[np.ix_(io, io)]
    return Dee - Deo @ np.linalg.solve(Doo, Doe)
