"""Python binding of libqxd (MI355X / gfx950): argument marshalling only.

Every function has the name of the C entry point it wraps (see
``include/qxd.h``) and forwards torch device tensors as raw pointers, with the
caller's current HIP stream.  All arithmetic runs in the library's HIP kernels;
there is no fallback: importing this module on a machine without the built
library or without a GPU raises.

Field tensors (device, contiguous) in the library's even-odd SoA layout:
``F64`` complex128, ``F32`` complex64, ``BF16`` bfloat16 (re, im pairs);
a half field holds 12 Ve complex numbers, a full field 24 Ve.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.environ.get("QXD_LIBRARY", os.path.join(_HERE, "libqxd.so"))

F64, F32, BF16 = 0, 1, 2
NN_NWEIGHTS = 207360

STATUS = {0: "QXD_OK", 1: "QXD_EINVAL", 2: "QXD_EGEOM", 3: "QXD_ENOMEM", 4: "QXD_ESINGULAR",
          5: "QXD_ENAN", 6: "QXD_ENOCONV", 7: "QXD_EHIP", 8: "QXD_ESTATE",
          9: "QXD_ESCRATCH", 10: "QXD_EIO"}


class QxdError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__("%s returned %s" % (where, STATUS.get(code, code)))


class qxd_geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int * 4), ("cstar", ctypes.c_int), ("t_antiperiodic", ctypes.c_int)]


class qxd_flavour(ctypes.Structure):
    _fields_ = [("qhat", ctypes.c_int), ("invqel", ctypes.c_double), ("kappa", ctypes.c_double),
                ("su3csw", ctypes.c_double), ("u1csw", ctypes.c_double)]


class qxd_clover_stats(ctypes.Structure):
    _fields_ = [("min_pivot", ctypes.c_double), ("max_norm", ctypes.c_double), ("n_singular", ctypes.c_int64)]


class qxd_solver_params(ctypes.Structure):
    _fields_ = [("nmx", ctypes.c_int), ("res", ctypes.c_double), ("inner_prec", ctypes.c_int),
                ("inner_res", ctypes.c_double), ("nkv", ctypes.c_int), ("max_outer", ctypes.c_int),
                ("check_every", ctypes.c_int), ("fallback_after", ctypes.c_int), ("sap_ncy", ctypes.c_int),
                ("sap_nmr", ctypes.c_int), ("sap_plain", ctypes.c_int), ("dfl_nc", ctypes.c_int)]


class qxd_solver_stats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("outer_it", ctypes.c_int), ("inner_it", ctypes.c_int),
                ("schur_applies", ctypes.c_int64), ("nn_applies", ctypes.c_int64),
                ("true_residual", ctypes.c_double), ("t_ms", ctypes.c_double), ("fell_back", ctypes.c_int),
                ("sap_applies", ctypes.c_int64)]


class qxd_train_params(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_double),
                ("beta1", ctypes.c_double), ("beta2", ctypes.c_double), ("eps", ctypes.c_double),
                ("holdout", ctypes.c_int), ("seed", ctypes.c_uint64), ("loss", ctypes.c_int)]


class qxd_train_stats(ctypes.Structure):
    _fields_ = [("loss_first", ctypes.c_double), ("loss_last", ctypes.c_double),
                ("holdout_loss", ctypes.c_double), ("t_ms", ctypes.c_double), ("steps", ctypes.c_int64)]


def _struct_dict(s):
    return {name: getattr(s, name) for name, _ in s._fields_}


QXD_MS_MAXSHIFT = 24  # most shifts of one multi-shift solve (include/qxd.h)
_P, _I, _D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
_SIGNATURES = {
    "qxd_status_string": ([_I], ctypes.c_char_p),
    "qxd_create": ([ctypes.POINTER(qxd_geom), ctypes.POINTER(_P)], _I),
    "qxd_destroy": ([_P], _I),
    "qxd_volume": ([_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)], _I),
    "qxd_trim": ([_P], _I),
    "qxd_set_gauge": ([_P, _P, _P, _I, _P], _I),
    "qxd_set_flavour": ([_P, ctypes.POINTER(qxd_flavour), _P], _I),
    "qxd_clover_build": ([_P, _P], _I),
    "qxd_clover_invert": ([_P, ctypes.POINTER(qxd_clover_stats), _P], _I),
    "qxd_dw_apply": ([_P, _I, _P, _P, _P], _I),
    "qxd_dw_eo_schur": ([_P, _I, _I, _P, _P, _P], _I),
    "qxd_dw_eo_schur_noalloc": ([_P, _I, _I, _P, _P, _P], _I),
    "qxd_eo_source": ([_P, _P, _P, _P], _I),
    "qxd_eo_reconstruct": ([_P, _P, _P, _P, _P], _I),
    "qxd_pack": ([_P, _I, _P, _P, _P], _I),
    "qxd_unpack": ([_P, _I, _P, _P, _P], _I),
    "qxd_solve_cg": ([_P, ctypes.POINTER(qxd_solver_params), _P, _P, ctypes.POINTER(qxd_solver_stats), _P], _I),
    "qxd_solve_fgcr": ([_P, ctypes.POINTER(qxd_solver_params), _P, _P, _P, ctypes.POINTER(qxd_solver_stats), _P],
                       _I),
    "qxd_solve_mscg": ([_P, ctypes.POINTER(qxd_solver_params), _I, ctypes.POINTER(_D), ctypes.POINTER(_P), _P,
                        ctypes.POINTER(qxd_solver_stats), _P], _I),
    "qxd_rational_apply": ([_P, ctypes.POINTER(qxd_solver_params), _D, _I, ctypes.POINTER(_D), ctypes.POINTER(_D),
                            _P, _P, ctypes.POINTER(qxd_solver_stats), _P], _I),
    "qxd_solve_fgcr_dfl": ([_P, ctypes.POINTER(qxd_solver_params), _P, _P, _P, ctypes.POINTER(qxd_solver_stats),
                            _P], _I),
    "qxd_dfl_create": ([_P, _I, ctypes.POINTER(_P)], _I),
    "qxd_dfl_destroy": ([_P], _I),
    "qxd_dfl_generate": ([_P, _P, _P, _I, _I, _I, _P], _I),
    "qxd_dfl_little": ([_P, _P, _P], _I),
    "qxd_dfl_apply": ([_P, _P, _I, _I, _I, _I, _P, _P, _P], _I),
    "qxd_dfl_basis": ([_P, _P, _I, _P, _P], _I),
    "qxd_dfl_little_get": ([_P, _P, _P], _I),
    "qxd_dfl_size": ([_P, ctypes.POINTER(_I), ctypes.POINTER(_I)], _I),
    "qxd_nn_create": ([_P, ctypes.POINTER(_P)], _I),
    "qxd_nn_destroy": ([_P], _I),
    "qxd_nn_set_weights": ([_P, _P], _I),
    "qxd_nn_set_skip": ([_P, _D], _I),
    "qxd_nn_get_weights": ([_P, _P], _I),
    "qxd_nn_save": ([_P, ctypes.c_char_p], _I),
    "qxd_nn_load": ([_P, ctypes.c_char_p], _I),
    "qxd_nn_apply": ([_P, _P, _P, _P, _P], _I),
    "qxd_sap_apply": ([_P, _I, _I, _I, _P, _P, _P], _I),
    "qxd_sap_apply_full": ([_P, _I, _I, _I, _P, _P, _P], _I),
    "qxd_nn_loss_grad": ([_P, _P, _P, _P, _I, _I, ctypes.POINTER(_D), _P, _P], _I),
    "qxd_nn_harvest": ([_P, _P, _I, _P, _P, ctypes.POINTER(_I), _P], _I),
    "qxd_nn_train": ([_P, _P, ctypes.POINTER(qxd_train_params), _P, _P, _I, ctypes.POINTER(qxd_train_stats), _P],
                     _I),
}

_lib = None


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libqxd.so, building it first if it is absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def _check(code, where):
    if code != 0:
        raise QxdError(code, where)


def _ptr(t):
    if t is None:
        return None
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return t.data_ptr()


def _stream(stream):
    if stream is not None:
        return stream
    import torch
    return torch.cuda.current_stream().cuda_stream


# ------------------------------------------------------------ entry points

def qxd_status_string(code):
    return load().qxd_status_string(int(code)).decode()


def qxd_create(L, cstar, t_antiperiodic=False):
    g = qxd_geom((ctypes.c_int * 4)(*[int(v) for v in L]), int(cstar), int(bool(t_antiperiodic)))
    h = _P()
    _check(load().qxd_create(ctypes.byref(g), ctypes.byref(h)), "qxd_create")
    return h


def qxd_destroy(h):
    _check(load().qxd_destroy(h), "qxd_destroy")


def qxd_trim(h):
    _check(load().qxd_trim(h), "qxd_trim")


def qxd_volume(h):
    V, Ve = ctypes.c_int64(), ctypes.c_int64()
    _check(load().qxd_volume(h, ctypes.byref(V), ctypes.byref(Ve)), "qxd_volume")
    return V.value, Ve.value


def qxd_set_gauge(h, U_phys, A_phys, stream=None):
    """U_phys (4, Vphys, 3, 3) complex128 and A_phys (4, Vphys) float64: torch device
    tensors or numpy host arrays."""
    on_dev = not isinstance(U_phys, np.ndarray)
    if not on_dev:
        U_phys = np.ascontiguousarray(U_phys, dtype=np.complex128)
        A_phys = np.ascontiguousarray(A_phys, dtype=np.float64)
    _check(load().qxd_set_gauge(h, _ptr(U_phys), _ptr(A_phys), int(on_dev), _stream(stream)), "qxd_set_gauge")


def qxd_set_flavour(h, qhat, invqel, kappa, su3csw, u1csw, stream=None):
    f = qxd_flavour(int(qhat), float(invqel), float(kappa), float(su3csw), float(u1csw))
    _check(load().qxd_set_flavour(h, ctypes.byref(f), _stream(stream)), "qxd_set_flavour")


def qxd_clover_build(h, stream=None):
    _check(load().qxd_clover_build(h, _stream(stream)), "qxd_clover_build")


def qxd_clover_invert(h, stream=None, check=True):
    st = qxd_clover_stats()
    code = load().qxd_clover_invert(h, ctypes.byref(st), _stream(stream))
    if check:
        _check(code, "qxd_clover_invert")
    d = _struct_dict(st)
    d["status"] = code
    return d


def qxd_dw_apply(h, prec, out, inp, stream=None):
    _check(load().qxd_dw_apply(h, int(prec), _ptr(out), _ptr(inp), _stream(stream)), "qxd_dw_apply")


def qxd_dw_eo_schur(h, prec, dagger, out_e, in_e, stream=None):
    _check(load().qxd_dw_eo_schur(h, int(prec), int(bool(dagger)), _ptr(out_e), _ptr(in_e), _stream(stream)),
           "qxd_dw_eo_schur")


def qxd_dw_eo_schur_noalloc(h, prec, dagger, out_e, in_e, stream=None):
    _check(load().qxd_dw_eo_schur_noalloc(h, int(prec), int(bool(dagger)), _ptr(out_e), _ptr(in_e),
                                          _stream(stream)), "qxd_dw_eo_schur_noalloc")


def qxd_eo_source(h, bhat_e, b, stream=None):
    _check(load().qxd_eo_source(h, _ptr(bhat_e), _ptr(b), _stream(stream)), "qxd_eo_source")


def qxd_eo_reconstruct(h, x, x_e, b, stream=None):
    _check(load().qxd_eo_reconstruct(h, _ptr(x), _ptr(x_e), _ptr(b), _stream(stream)), "qxd_eo_reconstruct")


def qxd_pack(h, prec, soa, aos, stream=None):
    _check(load().qxd_pack(h, int(prec), _ptr(soa), _ptr(aos), _stream(stream)), "qxd_pack")


def qxd_unpack(h, prec, aos, soa, stream=None):
    _check(load().qxd_unpack(h, int(prec), _ptr(aos), _ptr(soa), _stream(stream)), "qxd_unpack")


def solver_params(nmx=100000, res=1e-10, inner_prec=F32, inner_res=0.0, nkv=16, max_outer=100, check_every=4,
                  fallback_after=50, sap_ncy=0, sap_nmr=4, sap_plain=0, dfl_nc=0):
    return qxd_solver_params(int(nmx), float(res), int(inner_prec), float(inner_res), int(nkv), int(max_outer),
                             int(check_every), int(fallback_after), int(sap_ncy), int(sap_nmr), int(sap_plain),
                             int(dfl_nc))


def qxd_solve_cg(h, params, x, b, stream=None, check=True):
    st = qxd_solver_stats()
    code = load().qxd_solve_cg(h, ctypes.byref(params), _ptr(x), _ptr(b), ctypes.byref(st), _stream(stream))
    if check:
        _check(code, "qxd_solve_cg")
    d = _struct_dict(st)
    d["status"] = code
    return d


def qxd_solve_fgcr(h, params, net, x, b, stream=None, check=True):
    st = qxd_solver_stats()
    code = load().qxd_solve_fgcr(h, ctypes.byref(params), net, _ptr(x), _ptr(b), ctypes.byref(st),
                                 _stream(stream))
    if check:
        _check(code, "qxd_solve_fgcr")
    d = _struct_dict(st)
    d["status"] = code
    return d


def qxd_solve_mscg(h, params, shifts, xs, b_e, stream=None, check=True):
    """x_e[j] = (D_hat^+ D_hat + shifts[j])^-1 b_e for every shift (FP64 even half fields)."""
    n = len(shifts)
    st = qxd_solver_stats()
    sh = (_D * n)(*[float(v) for v in shifts])
    ptrs = (_P * n)(*[_ptr(x) for x in xs])
    code = load().qxd_solve_mscg(h, ctypes.byref(params), n, sh, ptrs, _ptr(b_e), ctypes.byref(st), _stream(stream))
    if check:
        _check(code, "qxd_solve_mscg")
    d = _struct_dict(st)
    d["status"] = code
    return d


def qxd_rational_apply(h, params, A, nu, mu, out_e, in_e, stream=None, check=True):
    """out_e = A prod_j (D_hat^+ D_hat + nu_j^2) / (D_hat^+ D_hat + mu_j^2) in_e (FP64 even half fields)."""
    n = len(nu)
    st = qxd_solver_stats()
    nu_c = (_D * n)(*[float(v) for v in nu])
    mu_c = (_D * n)(*[float(v) for v in mu])
    code = load().qxd_rational_apply(h, ctypes.byref(params), float(A), n, nu_c, mu_c, _ptr(out_e), _ptr(in_e),
                                     ctypes.byref(st), _stream(stream))
    if check:
        _check(code, "qxd_rational_apply")
    d = _struct_dict(st)
    d["status"] = code
    return d


QXD_DFL_MAXNS, QXD_DFL_MAXNC = 24, 32  # include/qxd.h


def qxd_solve_fgcr_dfl(h, params, dfl, x, b, stream=None, check=True):
    st = qxd_solver_stats()
    code = load().qxd_solve_fgcr_dfl(h, ctypes.byref(params), dfl, _ptr(x), _ptr(b), ctypes.byref(st),
                                     _stream(stream))
    if check:
        _check(code, "qxd_solve_fgcr_dfl")
    d = _struct_dict(st)
    d["status"] = code
    return d


def qxd_dfl_create(h, ns):
    d = _P()
    _check(load().qxd_dfl_create(h, int(ns), ctypes.byref(d)), "qxd_dfl_create")
    return d.value


def qxd_dfl_destroy(d):
    _check(load().qxd_dfl_destroy(d), "qxd_dfl_destroy")


def qxd_dfl_generate(h, d, v, nit, ncy, nmr, stream=None):
    _check(load().qxd_dfl_generate(h, d, _ptr(v), int(nit), int(ncy), int(nmr), _stream(stream)), "qxd_dfl_generate")


def qxd_dfl_little(h, d, stream=None):
    _check(load().qxd_dfl_little(h, d, _stream(stream)), "qxd_dfl_little")


def qxd_dfl_apply(h, d, nc, ncy, nmr, eo, out_e, in_e, stream=None):
    _check(load().qxd_dfl_apply(h, d, int(nc), int(ncy), int(nmr), int(eo), _ptr(out_e), _ptr(in_e), _stream(stream)),
           "qxd_dfl_apply")


def qxd_dfl_basis(h, d, k, out, stream=None):
    _check(load().qxd_dfl_basis(h, d, int(k), _ptr(out), _stream(stream)), "qxd_dfl_basis")


def qxd_dfl_size(d):
    nb, ns = _I(), _I()
    _check(load().qxd_dfl_size(d, ctypes.byref(nb), ctypes.byref(ns)), "qxd_dfl_size")
    return nb.value, ns.value


def qxd_dfl_little_get(d):
    """(A as complex64 [nblk][9][ns][ns], [block][n][k][l], and nbr [nblk][9]) on the host."""
    nblk, ns = qxd_dfl_size(d)
    A = np.zeros((nblk, 9, ns, ns), dtype=np.complex64)
    nbr = np.zeros((nblk, 9), dtype=np.int32)
    _check(load().qxd_dfl_little_get(d, A.ctypes.data, nbr.ctypes.data), "qxd_dfl_little_get")
    return A, nbr


def qxd_nn_create(h):
    net = _P()
    _check(load().qxd_nn_create(h, ctypes.byref(net)), "qxd_nn_create")
    return net


def qxd_nn_destroy(net):
    _check(load().qxd_nn_destroy(net), "qxd_nn_destroy")


def qxd_nn_set_skip(net, skip):
    _check(load().qxd_nn_set_skip(net, float(skip)), "qxd_nn_set_skip")


def qxd_nn_set_weights(net, w):
    w = np.ascontiguousarray(w, dtype=np.float32)
    assert w.size == NN_NWEIGHTS
    _check(load().qxd_nn_set_weights(net, w.ctypes.data), "qxd_nn_set_weights")


def qxd_nn_get_weights(net):
    w = np.empty(NN_NWEIGHTS, dtype=np.float32)
    _check(load().qxd_nn_get_weights(net, w.ctypes.data), "qxd_nn_get_weights")
    return w


def qxd_nn_save(net, path):
    _check(load().qxd_nn_save(net, os.fsencode(path)), "qxd_nn_save")


def qxd_nn_load(net, path):
    _check(load().qxd_nn_load(net, os.fsencode(path)), "qxd_nn_load")


def qxd_sap_apply(h, ncy, nmr, eo, out_e, in_e, stream=None):
    _check(load().qxd_sap_apply(h, int(ncy), int(nmr), int(eo), _ptr(out_e), _ptr(in_e), _stream(stream)),
           "qxd_sap_apply")


def qxd_sap_apply_full(h, ncy, nmr, eo, out, inp, stream=None):
    _check(load().qxd_sap_apply_full(h, int(ncy), int(nmr), int(eo), _ptr(out), _ptr(inp), _stream(stream)),
           "qxd_sap_apply_full")


def qxd_nn_apply(h, net, out_e, in_e, stream=None):
    _check(load().qxd_nn_apply(h, net, _ptr(out_e), _ptr(in_e), _stream(stream)), "qxd_nn_apply")


def qxd_nn_loss_grad(h, net, r, e, n, loss_kind=0, stream=None):
    loss = ctypes.c_double()
    g = np.empty(NN_NWEIGHTS, dtype=np.float32)
    _check(load().qxd_nn_loss_grad(h, net, _ptr(r), _ptr(e), int(n), int(loss_kind), ctypes.byref(loss),
                                   g.ctypes.data, _stream(stream)), "qxd_nn_loss_grad")
    return loss.value, g


def qxd_nn_harvest(h, b, npairs, r_out, e_out, stream=None):
    got = ctypes.c_int()
    _check(load().qxd_nn_harvest(h, _ptr(b), int(npairs), _ptr(r_out), _ptr(e_out), ctypes.byref(got),
                                 _stream(stream)), "qxd_nn_harvest")
    return got.value


def train_params(epochs=10, batch=8, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, holdout=0, seed=0, loss=1):
    return qxd_train_params(int(epochs), int(batch), float(lr), float(beta1), float(beta2), float(eps), int(holdout),
                            int(seed), int(loss))


def qxd_nn_train(h, net, params, r, e, npairs, stream=None):
    st = qxd_train_stats()
    _check(load().qxd_nn_train(h, net, ctypes.byref(params), _ptr(r), _ptr(e), int(npairs), ctypes.byref(st),
                               _stream(stream)), "qxd_nn_train")
    return _struct_dict(st)


# ------------------------------------------------------------ conveniences

def field(Ve, prec, full=False, zero=True):
    """A device field tensor of the given precision (half or full)."""
    import torch
    n = (24 if full else 12) * int(Ve)
    if prec == F64:
        t = torch.zeros(n, dtype=torch.complex128, device="cuda") if zero else torch.empty(
            n, dtype=torch.complex128, device="cuda")
    elif prec == F32:
        t = torch.zeros(n, dtype=torch.complex64, device="cuda") if zero else torch.empty(
            n, dtype=torch.complex64, device="cuda")
    elif prec == BF16:
        t = torch.zeros(2 * n, dtype=torch.bfloat16, device="cuda") if zero else torch.empty(
            2 * n, dtype=torch.bfloat16, device="cuda")
    else:
        raise ValueError(prec)
    return t


class Lattice:
    """Owns one qxd handle."""

    def __init__(self, L, cstar, t_antiperiodic=False):
        self.L = tuple(L)
        self.cstar = cstar
        self.h = qxd_create(L, cstar, t_antiperiodic)
        self.V, self.Ve = qxd_volume(self.h)

    def close(self):
        if self.h:
            qxd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, U_phys, A_phys, flavour):
        qxd_set_gauge(self.h, U_phys, A_phys)
        qxd_set_flavour(self.h, **flavour)
        qxd_clover_build(self.h)
        return qxd_clover_invert(self.h)

    def field(self, prec, full=False, zero=True):
        return field(self.Ve, prec, full, zero)

    def pack(self, aos, prec=F64):
        """Canonical (V, 4, 3) complex128 device tensor -> full eo field."""
        out = self.field(prec, full=True, zero=False)
        qxd_pack(self.h, prec, out, aos.contiguous())
        return out

    def unpack(self, soa, prec=F64):
        import torch
        out = torch.empty((self.V, 4, 3), dtype=torch.complex128, device="cuda")
        qxd_unpack(self.h, prec, out, soa)
        return out
