"""Host-side checks of the C ABI that need no GPU: the library loads,
exports every function declared in include/paulinet.h, and rejects bad
arguments before touching the device."""

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "paulinet.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(pn_[a-z_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_expected_entry_points():
    names = declared_functions()
    for n in ("pn_ctx_create", "pn_ctx_destroy", "pn_param_count", "pn_workspace_bytes", "pn_eval",
              "pn_eval_backward", "pn_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1909_08423_amd as pn
    path = pn.library_path()
    if not os.path.exists(path):
        pytest.skip("library not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(path)
    for n in declared_functions():
        assert hasattr(lib, n), f"{n} not exported"


def test_status_strings_and_argument_validation():
    import paper_1909_08423_amd as pn
    from paper_1909_08423_amd._lib import pn_net_desc, pn_system_desc
    if not os.path.exists(pn.library_path()):
        pytest.skip("library not built")
    lib = pn.load_library()
    assert lib.pn_status_string(0) == b"ok"
    assert lib.pn_status_string(4) == b"workspace too small"
    out = ctypes.c_void_p(1)
    # null descriptions are rejected before any device call
    assert lib.pn_ctx_create(None, None, ctypes.byref(out)) == 1
    assert out.value is None
    s = pn_system_desc()
    n = pn_net_desc()
    assert lib.pn_ctx_create(ctypes.byref(s), ctypes.byref(n), ctypes.byref(out)) == 1
    # unsupported shapes (d-shell) are refused before any device call
    keep = []

    def arr(a, dt):
        a = np.ascontiguousarray(a, dtype=dt)
        keep.append(a)
        return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double if dt == np.float64 else ctypes.c_int32))

    s.n_nuc = 1
    s.nuc_xyz = arr([0.0, 0, 0], np.float64)
    s.charge = arr([1.0], np.float64)
    s.n_up, s.n_down = 1, 0
    s.n_shell = 1
    s.shell_center = arr([0], np.int32)
    s.shell_l = arr([2], np.int32)
    s.shell_exp = arr([1.0], np.float64)
    s.n_mo = 1
    s.mo_coeff = arr(np.ones(5), np.float64)
    s.n_det = 1
    s.det_up = arr([0], np.int32)
    s.det_down = arr([0], np.int32)
    s.ci = arr([1.0], np.float64)
    n.n_feat, n.feat_cutoff, n.dim_x, n.dim_z, n.n_layers = 16, 10.0, 16, 16, 1
    assert lib.pn_ctx_create(ctypes.byref(s), ctypes.byref(n), ctypes.byref(out)) == 2
    # out-of-range determinant orbital index
    s.shell_l = arr([0], np.int32)
    s.det_up = arr([3], np.int32)
    assert lib.pn_ctx_create(ctypes.byref(s), ctypes.byref(n), ctypes.byref(out)) == 1
    # too many layers; widths the matrix-core products do not take
    s.det_up = arr([0], np.int32)
    n.n_layers = 99
    assert lib.pn_ctx_create(ctypes.byref(s), ctypes.byref(n), ctypes.byref(out)) == 2
    n.n_layers = 1
    n.dim_x = 48
    assert lib.pn_ctx_create(ctypes.byref(s), ctypes.byref(n), ctypes.byref(out)) == 2
    # a null context is an invalid argument for every call
    assert lib.pn_eval(None, None, 1, None, None, 0, None, None, None, None, None, None, 0) == 1
    assert lib.pn_param_count(None) == -1
