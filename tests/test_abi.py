"""The C-ABI library loads and exports every entry point include/ptp.h
declares; host-side argument checks (no GPU needed)."""
import ctypes as C
import os
import re

import pytest

import paper_1810_08218_amd as P
from paper_1810_08218_amd import ptp as B

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ptp.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ptp_[a-z0-9_]+)\s*\(", txt)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(B.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = P.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert lib.ptp_version().startswith(b"ptp-mi355x")


@pytest.mark.parametrize("n,f,m,tol", [(0, 0, 1, 1e-3), (10, -1, 1, 1e-3), (10, 4, 0, 1e-3),
                                       (10, 4, 11, 1e-3), (10, 4, 1, 0.0), (10, 4, 1, -1.0)])
def test_plan_rejects_bad_sizes(n, f, m, tol):
    with pytest.raises(P.PTPError) as e:
        P.Plan(n, f, m, tol)
    assert e.value.status == P.PTP_EINVAL


@pytest.mark.parametrize("n,f", [((1 << 29) + 1, 4), (10, (1 << 31) // 6 + 1)])
def test_plan_rejects_unsupported_sizes(n, f):
    with pytest.raises(P.PTPError) as e:
        P.Plan(n, f, 1, 1e-3)
    assert e.value.status == P.PTP_EUNSUPPORTED


def test_null_plan_calls_are_einval():
    lib = P.load()
    assert lib.ptp_workspace_bytes(None, None) == P.PTP_EINVAL
    assert lib.ptp_prepare(None, None, None, None, None, 0, None) == P.PTP_EINVAL
    assert lib.ptp_run(None, None, None, None) == P.PTP_EINVAL
    assert lib.ptp_get_stats(None, None) == P.PTP_EINVAL
    assert lib.ptp_n_toplesets(None) == -1
    assert lib.ptp_last_error(None) == b"null plan"
    out = C.c_void_p(1)
    assert lib.ptp_plan_create(C.byref(out), 0, 0, 1, None) == P.PTP_EINVAL
    assert out.value is None
