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


def extended_from_physical(o, f_phys, mirror):
    """A physical-lattice site field extended to the extended lattice: the
    mirror half x1 >= L1 holds mirror(f) of the site x1 - L1."""
    x = o.coords(np.arange(o.V))
    m = x[:, 1] >= o.L[1]
    x1 = np.where(m, x[:, 1] - o.L[1], x[:, 1])
    sp = x[:, 3] + o.L[3] * (x[:, 2] + o.L[2] * (x1 + o.L[1] * x[:, 0]))
    f = f_phys[sp].copy()
    f[m] = mirror(f[m])
    return f


def gauge_rotate(o, U_phys, A_phys, qhat, seed):
    """A random gauge transformation (Omega(x) in SU(3), alpha(x) real, with
    the C* constraint Omega(x + L1 e1) = Omega(x)*, alpha -> -alpha on the
    mirror half) applied to physical fields: U'(x,mu) = Omega(x) U(x,mu)
    Omega(x+mu)^+, A'(x,mu) = A(x,mu) + alpha(x) - alpha(x+mu), with x + mu
    taken on the extended lattice.  Returns (U', A', g) where g(x) =
    Omega(x) exp(i qhat alpha(x)) acts on the colour index of a spinor at every
    extended site (D' = g D g^-1 for that charge)."""
    om = extended_from_physical(o, sg.transform_su3(seed, 1.0, o.Vphys), np.conj)
    al = extended_from_physical(o, sg.angles(seed + 1, 1.0, o.Vphys), np.negative)
    nb, _ = o.neighbours()
    x = o.coords(np.arange(o.V))
    phys = np.nonzero(x[:, 1] < o.L[1])[0]  # extended index of every physical site, in physical order
    U = np.asarray(U_phys).reshape(4, o.Vphys, 3, 3)
    A = np.asarray(A_phys).reshape(4, o.Vphys)
    U2 = np.empty_like(U)
    A2 = np.empty_like(A)
    for mu in range(4):
        fw = nb[phys, mu, 0]
        U2[mu] = om[phys] @ U[mu] @ np.conj(np.swapaxes(om[fw], 1, 2))
        A2[mu] = A[mu] + al[phys] - al[fw]
    g = om * np.exp(1j * qhat * al)[:, None, None]
    return U2, A2, g


def rotate_spinor(g, psi):
    """psi'(x) = g(x) psi(x) on the colour index (spinor shape (V, 4, 3))."""
    return np.einsum("vab,vsb->vsa", g, psi)
