"""Shared set-up of the GPU parity tests: the same seeded inputs go to the oracle
(CPU, FP64) and to libqxd (GPU) through its C ABI."""
import numpy as np

import oracle
import synthgen as sg


def rel_err(got, want):
    """max |got - want| / max |want| over all components."""
    return float(np.abs(got - want).max() / max(np.abs(want).max(), 1e-300))


def norm_err(got, want):
    return float(np.linalg.norm(got - want) / np.linalg.norm(want))


def make_pair(L, cstar, flav, sigma=0.2, su1=0.3, seed=7, tanti=False, cache=True):
    import torch  # noqa: F401
    import paper_1908_11673_amd as qxd
    o = oracle.Oracle(L, cstar, tanti)
    U = sg.gauge_su3(seed, sigma, o.Vphys)
    A = sg.gauge_u1(seed, su1, o.Vphys)
    o.set_gauge_physical(U, A)
    o.set_flavour(**flav, cache=cache)
    lat = qxd.Lattice(L, cstar, tanti)
    stats = lat.setup(U, A, flav)
    return o, lat, stats


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def even_only(o, psi):
    out = psi.copy()
    out[o.parity() == 1] = 0
    return out


def half32(lat, psi):
    """even-site spinor (V, 4, 3) -> FP32 even half field on the device"""
    import paper_1908_11673_amd as qxd
    return lat.pack(to_dev(psi), qxd.F32)[:12 * lat.Ve].clone()


def from_half32(lat, t):
    """FP32 even half field -> (V, 4, 3) complex128 spinor (odd sites zero)"""
    import paper_1908_11673_amd as qxd
    full = lat.field(qxd.F32, full=True)
    full[:12 * lat.Ve] = t
    return lat.unpack(full, qxd.F32).cpu().numpy()


def half64(lat, psi):
    """even-site spinor (V, 4, 3) -> FP64 even half field on the device"""
    import paper_1908_11673_amd as qxd
    return lat.pack(to_dev(psi), qxd.F64)[:12 * lat.Ve].clone()


def from_half64(lat, t):
    """FP64 even half field -> (V, 4, 3) complex128 spinor (odd sites zero)"""
    import paper_1908_11673_amd as qxd
    full = lat.field(qxd.F64, full=True)
    full[:12 * lat.Ve] = t
    return lat.unpack(full, qxd.F64).cpu().numpy()
