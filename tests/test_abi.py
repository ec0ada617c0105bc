"""The C ABI library loads on a machine without a GPU, exports every entry point
that include/qxd.h declares, and rejects bad geometry on the host before any
device call."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    txt = open(os.path.join(ROOT, "include", "qxd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(qxd_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_the_hot_path_calls():
    names = declared_entry_points()
    for n in ("qxd_dw_apply", "qxd_dw_eo_schur", "qxd_clover_build", "qxd_clover_invert", "qxd_solve_cg",
              "qxd_solve_fgcr", "qxd_eo_source", "qxd_eo_reconstruct", "qxd_nn_apply", "qxd_nn_train"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1908_11673_amd as qxd
    qxd.load()  # builds the library when it is absent (fresh checkout)
    lib = ctypes.CDLL(qxd.lib_path())
    missing = [n for n in declared_entry_points() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_wraps_every_declared_symbol():
    import paper_1908_11673_amd as qxd
    missing = [n for n in declared_entry_points() if not hasattr(qxd, n)]
    assert not missing, missing


@pytest.mark.parametrize("L,cstar", [((4, 3, 4, 4), 1), ((4, 4, 4, 4), 4), ((4, 4, 4, 4), -1), ((0, 4, 4, 4), 0),
                                     ((2048, 1024, 1024, 2), 1)])
def test_bad_geometry_is_rejected_on_the_host(L, cstar):
    import paper_1908_11673_amd as qxd
    with pytest.raises(qxd.QxdError) as e:
        qxd.qxd_create(L, cstar)
    assert e.value.code == 2


def test_status_strings():
    import paper_1908_11673_amd as qxd
    lib = qxd.load()
    assert lib.qxd_status_string(0) == b"QXD_OK"
    assert lib.qxd_status_string(4) == b"QXD_ESINGULAR"
