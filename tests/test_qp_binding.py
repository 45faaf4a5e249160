"""Host-side checks of the Algorithm 1 binding (no GPU): the options and
result structures match the C header, defaults are the documented ones,
and malformed patterns are refused before any device work."""
import ctypes as C
import re
import os

import numpy as np
import pytest

from paper_2510_05885_amd import ncl_kkt as nk

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _fields(struct_name):
    hdr = open(os.path.join(ROOT, "include", "ncl_kkt.h")).read()
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + struct_name + ";", hdr).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return [m.group(2) for m in re.finditer(r"(int32_t|double)\s+(\w+);", body)]


def test_structures_match_the_header():
    assert [f[0] for f in nk.QpOptions._fields_] == _fields("ncl_qp_options")
    assert [f[0] for f in nk.QpResult._fields_] == _fields("ncl_qp_result")


def test_default_options():
    o = nk.QpOptions()
    nk.lib().ncl_qp_default_options(C.byref(o))
    assert (o.eta_star, o.omega_star, o.max_outer, o.max_inner, o.precision, o.print_level) == \
        (1e-8, 1e-8, 100, 100, nk.NCL_FP64, 0)


def test_bad_arguments_are_refused_on_the_host():
    o = nk.QpOptions()
    L = nk.lib()
    L.ncl_qp_default_options(C.byref(o))
    res = nk.QpResult()
    qc, qcp = nk._i32([0, 1])
    qr, qrp = nk._i32([0])
    dummy = C.c_void_p(8)   # never dereferenced: every call below fails its argument checks first
    # n < 1
    assert L.ncl_qp_solve(C.byref(o), 0, 0, qcp, qrp, dummy, dummy, None, None, None, None, dummy, dummy,
                          dummy, dummy, dummy, dummy, C.byref(res), None) == nk.NCL_ERR_ARG
    # m > 0 without A
    assert L.ncl_qp_solve(C.byref(o), 1, 1, qcp, qrp, dummy, dummy, None, None, None, None, dummy, dummy,
                          dummy, dummy, dummy, dummy, C.byref(res), None) == nk.NCL_ERR_ARG
    # non-positive tolerance
    o.eta_star = 0.0
    assert L.ncl_qp_solve(C.byref(o), 1, 0, qcp, qrp, dummy, dummy, None, None, None, None, dummy, dummy,
                          dummy, dummy, dummy, dummy, C.byref(res), None) == nk.NCL_ERR_ARG
