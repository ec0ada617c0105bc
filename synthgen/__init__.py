"""Seeded synthetic inputs shared by the GPU path and the oracle.

Holds none of the method's arithmetic: only counter-based random numbers
(Philox-4x32-10), Gaussian deviates, random SU(3) links (exp of a Gaussian
traceless anti-Hermitian matrix, projected back onto SU(3)), U(1) angles and
Gaussian complex spinors.  The generator is in ``synth.c``; this module is its
ctypes wrapper and returns numpy arrays.

Layouts (complex128 unless stated):

* SU(3) links on a list of sites: ``(4, n, 3, 3)``, index ``[mu][k][row][col]``.
* U(1) angles: float64 ``(4, n)``.
* Spinors: ``(n, 4, 3)``, index ``[k][spin][colour]``.

Site ``k`` means canonical index ``idx[k]`` when a list is passed, else ``k``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64, U64, D, U32 = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_uint32
        lib.sg_philox4x32_10.argtypes = [P, P, P]
        for name in ("sg_gauge_su3", "sg_transform_su3"):
            getattr(lib, name).argtypes = [U64, D, P, I64, P]
        lib.sg_gauge_u1.argtypes = [U64, D, P, I64, P]
        lib.sg_angle.argtypes = [U64, D, P, I64, P]
        lib.sg_spinor.argtypes = [U64, P, I64, P]
        lib.sg_gaussian.argtypes = [U64, U32, D, I64, P]
        _lib = lib
    return _lib


def _idx(sites):
    if isinstance(sites, (int, np.integer)):
        return None, int(sites)
    idx = np.ascontiguousarray(np.asarray(sites, dtype=np.int64))
    return idx, int(idx.size)


def _ptr(a):
    return None if a is None else a.ctypes.data


def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(ctr, dtype=np.uint32))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint32))
    out = np.zeros(4, dtype=np.uint32)
    _load().sg_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def gauge_su3(seed: int, sigma: float, sites) -> np.ndarray:
    """SU(3) links U[mu][k] for ``sites`` (a count or a list of canonical indices)."""
    idx, n = _idx(sites)
    out = np.empty((4, n, 3, 3), dtype=np.complex128)
    _load().sg_gauge_su3(seed, sigma, _ptr(idx), n, _ptr(out))
    return out


def gauge_u1(seed: int, sigma: float, sites) -> np.ndarray:
    idx, n = _idx(sites)
    out = np.empty((4, n), dtype=np.float64)
    _load().sg_gauge_u1(seed, sigma, _ptr(idx), n, _ptr(out))
    return out


def spinor(seed: int, sites) -> np.ndarray:
    idx, n = _idx(sites)
    out = np.empty((n, 4, 3), dtype=np.complex128)
    _load().sg_spinor(seed, _ptr(idx), n, _ptr(out))
    return out


def transform_su3(seed: int, sigma: float, sites) -> np.ndarray:
    idx, n = _idx(sites)
    out = np.empty((n, 3, 3), dtype=np.complex128)
    _load().sg_transform_su3(seed, sigma, _ptr(idx), n, _ptr(out))
    return out


def angles(seed: int, sigma: float, sites) -> np.ndarray:
    idx, n = _idx(sites)
    out = np.empty(n, dtype=np.float64)
    _load().sg_angle(seed, sigma, _ptr(idx), n, _ptr(out))
    return out


def gaussian(seed: int, tag: int, sigma: float, n: int) -> np.ndarray:
    out = np.empty(int(n), dtype=np.float64)
    _load().sg_gaussian(seed, tag, sigma, int(n), _ptr(out))
    return out


# Workload recipes (lattice extents are physical L0, L1, L2, L3; time first).
WORKLOADS = {
    "c0": dict(L=(8, 4, 4, 4), cstar=1, sigma_su3=0.2, sigma_u1=0.3, gauge_seed=0, source_seed=1000),
    "c1": dict(L=(64, 32, 32, 32), cstar=3, sigma_su3=0.2, sigma_u1=0.3, gauge_seed=1, source_seed=1100),
    "c2": dict(L=(48, 24, 24, 24), cstar=3, sigma_su3=0.3, sigma_u1=0.3, gauge_seed=2, source_seed=2000),
    "c3": dict(L=(32, 16, 16, 16), cstar=3, sigma_su3=0.2, sigma_u1=0.3, gauge_seed=3000, source_seed=3500),
    "c4": dict(L=(128, 64, 64, 64), cstar=3, sigma_su3=0.2, sigma_u1=0.3, gauge_seed=4, source_seed=4000),
}

# Flavour parameters of the sample run (down-type and up-type quark).
FLAVOURS = {
    "d": dict(qhat=-2, invqel=6.0, kappa=0.136377, su3csw=1.909520, u1csw=1.0),
    "u": dict(qhat=4, invqel=6.0, kappa=0.137312, su3csw=1.909520, u1csw=1.0),
}
