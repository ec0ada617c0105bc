"""FP64 CPU oracle for the Wilson-clover / C* hot path (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU path.
The arithmetic is in ``qxd_oracle.c`` (plain C, FP64, no FMA contraction);
this module wraps it with ctypes and adds the network composition
(``oracle.nn``) and dense-matrix tools for tiny lattices (``oracle.dense``).

Every field is on the extended lattice in the canonical layout:
spinors ``(V, 4, 3)`` complex128 indexed by the site
``x3 + L3 (x2 + L2 (x1 + L1ext x0))``; links ``(4, V, 3, 3)``; angles
``(4, V)``.  Even-site vectors are full-lattice arrays whose odd sites are
ignored on input and zero on output.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "qxd_oracle.c")
_LIB = os.path.join(_HERE, "libqxd_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc: -O2, no FMA contraction, OpenMP; complex
    arithmetic by the textbook formulas (-fcx-limited-range).  For products of
    finite operands that is the value C99's Annex G gives, without a library
    call per product.  Complex divisions (the pivoting in the 6x6 block
    solves) lose Annex G's range reduction: a|b|^2 may round differently, which
    changes results at the level of a few ulp, and would overflow or underflow
    only for entries beyond about 1e154 or below 1e-154, far outside any field
    here."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fcx-limited-range", "-fPIC",
                        "-shared", "-fopenmp", "-std=c11", "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P, I, I64, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_double
        sig = {
            "or_create": ([I, I, I, I, I, I], P),
            "or_destroy": ([P], None),
            "or_volume": ([P], I64),
            "or_extents": ([P, P], None),
            "or_neighbours": ([P, P, P], None),
            "or_shift": ([P, I64, P], I64),
            "or_parity": ([P, P], None),
            "or_set_gauge_physical": ([P, P, P], None),
            "or_set_gauge_extended": ([P, P, P], None),
            "or_get_gauge_extended": ([P, P, P], None),
            "or_set_flavour": ([P, I, D, D, D, D, I], None),
            "or_cache_blocks": ([P], None),
            "or_field_tensors": ([P, I64, P, P], None),
            "or_sw_site": ([P, I64, P], None),
            "or_dirac": ([P, P, P], None),
            "or_dirac_sites": ([P, P, P, I64, P], None),
            "or_site_block": ([P, I64, P], None),
            "or_schur": ([P, P, P, I], None),
            "or_schur_sites": ([P, P, P, I64, P, I], None),
            "or_min_block_pivot": ([P], D),
            "or_eo_source": ([P, P, P], None),
            "or_eo_reconstruct": ([P, P, P, P], None),
            "or_cg": ([P, P, P, D, I, P], I),
            "or_nn_conv": ([P, I, I, P, P, P], None),
            "or_nn_conv_adjoint": ([P, I, I, P, P, P], None),
            "or_nn_conv_wgrad": ([P, I, I, P, P, P], None),
        }
        for name, (args, res) in sig.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


class Oracle:
    """Extended lattice of physical extents ``L = (L0, L1, L2, L3)``."""

    def __init__(self, L, cstar: int, t_antiperiodic: bool = False):
        self._lib = _load()
        self.L = tuple(int(v) for v in L)
        self.cstar = int(cstar)
        self.h = self._lib.or_create(*self.L, self.cstar, int(bool(t_antiperiodic)))
        if not self.h:
            raise ValueError("invalid geometry %r cstar=%d" % (L, cstar))
        self.V = int(self._lib.or_volume(self.h))
        le = np.zeros(4, dtype=np.int32)
        self._lib.or_extents(self.h, le.ctypes.data)
        self.Le = tuple(int(v) for v in le)
        self.Vphys = self.L[0] * self.L[1] * self.L[2] * self.L[3]
        self._has_gauge = False
        self._has_flavour = False

    def _need(self, flavour=True):
        # the C side dereferences the links (and the flavour's tables) unchecked
        if not self._has_gauge or (flavour and not self._has_flavour):
            raise RuntimeError("oracle: set the gauge field%s first" % (" and the flavour" if flavour else ""))

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._lib.or_destroy(h)
            self.h = None

    # geometry
    def neighbours(self):
        nb = np.empty((self.V, 4, 2), dtype=np.int64)
        sg = np.empty((self.V, 4, 2), dtype=np.float64)
        self._lib.or_neighbours(self.h, nb.ctypes.data, sg.ctypes.data)
        return nb, sg

    def parity(self):
        p = np.empty(self.V, dtype=np.int8)
        self._lib.or_parity(self.h, p.ctypes.data)
        return p

    def shift(self, site: int, d) -> int:
        dd = _c(d, np.int32)
        return int(self._lib.or_shift(self.h, int(site), dd.ctypes.data))

    def coords(self, site):
        s = np.asarray(site, dtype=np.int64)
        x3 = s % self.Le[3]; s = s // self.Le[3]
        x2 = s % self.Le[2]; s = s // self.Le[2]
        x1 = s % self.Le[1]; x0 = s // self.Le[1]
        return np.stack([x0, x1, x2, x3], axis=-1)

    def site(self, x):
        x = np.asarray(x, dtype=np.int64)
        return x[..., 3] + self.Le[3] * (x[..., 2] + self.Le[2] * (x[..., 1] + self.Le[1] * x[..., 0]))

    # gauge
    def set_gauge_physical(self, U, A):
        U = _c(U, np.complex128)
        A = _c(A, np.float64)
        assert U.shape == (4, self.Vphys, 3, 3) and A.shape == (4, self.Vphys)
        self._lib.or_set_gauge_physical(self.h, U.ctypes.data, A.ctypes.data)
        self._has_gauge = True

    def set_gauge_extended(self, U, A):
        U = _c(U, np.complex128)
        A = _c(A, np.float64)
        assert U.shape == (4, self.V, 3, 3) and A.shape == (4, self.V)
        self._lib.or_set_gauge_extended(self.h, U.ctypes.data, A.ctypes.data)
        self._has_gauge = True

    def gauge_extended(self):
        self._need(flavour=False)
        U = np.empty((4, self.V, 3, 3), dtype=np.complex128)
        A = np.empty((4, self.V), dtype=np.float64)
        self._lib.or_get_gauge_extended(self.h, U.ctypes.data, A.ctypes.data)
        return U, A

    def set_flavour(self, qhat, invqel, kappa, su3csw, u1csw, cache=True, blocks=None):
        self._need(flavour=False)
        self._lib.or_set_flavour(self.h, int(qhat), float(invqel), float(kappa), float(su3csw),
                                 float(u1csw), int(bool(cache)))
        self._has_flavour = True
        if blocks if blocks is not None else cache:
            self._lib.or_cache_blocks(self.h)

    # operator
    def _spinor(self, psi):
        psi = _c(psi, np.complex128)
        assert psi.shape == (self.V, 4, 3), psi.shape
        return psi

    def field_tensors(self, site: int):
        self._need(flavour=False)
        F = np.empty((4, 4, 3, 3), dtype=np.complex128)
        A = np.empty((4, 4), dtype=np.complex128)
        self._lib.or_field_tensors(self.h, int(site), F.ctypes.data, A.ctypes.data)
        return F, A

    def sw_site(self, site: int):
        self._need()
        M = np.empty((12, 12), dtype=np.complex128)
        self._lib.or_sw_site(self.h, int(site), M.ctypes.data)
        return M

    def site_block(self, site: int):
        self._need()
        M = np.empty((12, 12), dtype=np.complex128)
        self._lib.or_site_block(self.h, int(site), M.ctypes.data)
        return M

    def dirac(self, psi):
        self._need()
        psi = self._spinor(psi)
        out = np.empty_like(psi)
        self._lib.or_dirac(self.h, psi.ctypes.data, out.ctypes.data)
        return out

    def dirac_sites(self, psi, sites):
        self._need()
        psi = self._spinor(psi)
        s = _c(sites, np.int64)
        out = np.empty((s.size, 4, 3), dtype=np.complex128)
        self._lib.or_dirac_sites(self.h, psi.ctypes.data, s.ctypes.data, s.size, out.ctypes.data)
        return out

    def schur(self, psi, dagger=False):
        self._need()
        psi = self._spinor(psi)
        out = np.empty_like(psi)
        self._lib.or_schur(self.h, psi.ctypes.data, out.ctypes.data, int(bool(dagger)))
        return out

    def schur_sites(self, psi, sites, dagger=False):
        self._need()
        psi = self._spinor(psi)
        s = _c(sites, np.int64)
        out = np.empty((s.size, 4, 3), dtype=np.complex128)
        self._lib.or_schur_sites(self.h, psi.ctypes.data, s.ctypes.data, s.size, out.ctypes.data,
                                 int(bool(dagger)))
        return out

    def min_block_pivot(self) -> float:
        self._need()
        return float(self._lib.or_min_block_pivot(self.h))

    def eo_source(self, b):
        self._need()
        b = self._spinor(b)
        out = np.empty_like(b)
        self._lib.or_eo_source(self.h, b.ctypes.data, out.ctypes.data)
        return out

    def eo_reconstruct(self, xe, b):
        self._need()
        xe = self._spinor(xe)
        b = self._spinor(b)
        out = np.empty_like(b)
        self._lib.or_eo_reconstruct(self.h, xe.ctypes.data, b.ctypes.data, out.ctypes.data)
        return out

    def cg(self, bhat, tol_abs, nmx=100000):
        self._need()
        bhat = self._spinor(bhat)
        x = np.empty_like(bhat)
        res = ctypes.c_double(0.0)
        it = self._lib.or_cg(self.h, bhat.ctypes.data, x.ctypes.data, float(tol_abs), int(nmx),
                             ctypes.byref(res))
        return x, int(it), float(res.value)

    # network layers
    def nn_conv(self, W, h):
        W = _c(W, np.float64)
        h = _c(h, np.float64)
        cout, cin = W.shape[1], W.shape[2]
        assert W.shape == (81, cout, cin) and h.shape == (self.V, cin)
        y = np.empty((self.V, cout), dtype=np.float64)
        self._lib.or_nn_conv(self.h, cin, cout, W.ctypes.data, h.ctypes.data, y.ctypes.data)
        return y

    def nn_conv_adjoint(self, W, g):
        W = _c(W, np.float64)
        g = _c(g, np.float64)
        cout, cin = W.shape[1], W.shape[2]
        dh = np.empty((self.V, cin), dtype=np.float64)
        self._lib.or_nn_conv_adjoint(self.h, cin, cout, W.ctypes.data, g.ctypes.data, dh.ctypes.data)
        return dh

    def nn_conv_wgrad(self, g, h, cin, cout):
        g = _c(g, np.float64)
        h = _c(h, np.float64)
        dW = np.empty((81, cout, cin), dtype=np.float64)
        self._lib.or_nn_conv_wgrad(self.h, cin, cout, g.ctypes.data, h.ctypes.data, dW.ctypes.data)
        return dW
