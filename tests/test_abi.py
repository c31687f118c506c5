"""Host-side checks of the C ABI that need no GPU."""
import ctypes as C
import os
import re

import pytest

from paper_1908_02461_amd import atsfft as A

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "atsfft.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(atsfft_\w+)\s*\(", src, flags=re.M)))


def test_header_and_binding_agree():
    assert sorted(A.EXPORTS) == _declared()


def test_library_exports_every_declared_symbol():
    lib = A.load()
    for name in _declared():
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    lib = A.load()
    assert b"gfx950" in lib.atsfft_version()
    for s in range(6):
        assert lib.atsfft_status_string(s)
    assert lib.atsfft_status_string(99) == b"unknown status"


def test_default_desc_values():
    d = A.default_desc(1, 1 << 22, "c64")
    assert (d.B0, d.B_max, d.alpha_probe, d.alpha) == (32, 16384, 16, 32)
    assert (d.L_loc, d.L_est, d.T_vote, d.P_max, d.d, d.gamma) == (9, 9, 5, 12, 2, 32)
    assert d.delta == 1e-6
    d = A.default_desc(1, 1 << 14, "c128")
    assert d.B_max == 512 and d.delta == 1e-8
    d = A.default_desc(2, 4096, "c64")
    assert (d.B0, d.B_max, d.alpha, d.alpha_probe) == (8, 128, 8, 4)


@pytest.mark.parametrize("knobs", [
    dict(n=1000), dict(L_est=8), dict(L_est=33), dict(T_vote=0), dict(T_vote=10), dict(B0=48),
    dict(B0=64, B_max=32), dict(delta=0.0), dict(alpha=7), dict(max_out=0), dict(max_out=1 << 20),
    dict(P_max=0), dict(B_max=1 << 15), dict(q=1.0), dict(n=1 << 31), dict(ndim=3),
    dict(res_tol=-1.0), dict(res_retries=8), dict(res_retries=-1),
])
def test_plan_rejects_invalid_descriptors(knobs):
    lib = A.load()
    d = A.default_desc(1, 1 << 16, "c64")
    for k, v in knobs.items():
        setattr(d, k, v)
    h = C.c_void_p()
    assert lib.atsfft_plan(C.byref(h), C.byref(d)) == A.EINVAL
    assert not h.value
    assert lib.atsfft_last_error()


def test_fixed_b_validation():
    lib = A.load()
    d = A.default_desc(1, 1 << 16, "c64", fixed_B=3000)
    h = C.c_void_p()
    assert lib.atsfft_plan(C.byref(h), C.byref(d)) == A.EINVAL
    # re-runs of the residual test grow a fixed B up to B_max, which must be valid
    d = A.default_desc(1, 1 << 16, "c64", fixed_B=256, fixed_k=8, res_tol=1e-3, B_max=3000)
    assert lib.atsfft_plan(C.byref(h), C.byref(d)) == A.EINVAL


def test_descriptor_layout_matches_the_library():
    """atsfft_default_desc writes exactly sizeof(atsfft_desc) bytes: none past
    the binding's structure, and every field the binding declares."""
    lib = A.load()
    n = C.sizeof(A.Desc)
    buf = (C.c_uint8 * (n + 64))(*([0xA5] * (n + 64)))
    assert lib.atsfft_default_desc(C.cast(buf, C.POINTER(A.Desc)), 1, 1 << 16, A.C64) == A.SUCCESS
    assert bytes(buf[n:]) == b"\xa5" * 64
    d = C.cast(buf, C.POINTER(A.Desc)).contents
    assert d.res_tol == 0.0 and d.res_retries == 1 and d.n == 1 << 16


def test_graph_excludes_profile():
    lib = A.load()
    d = A.default_desc(1, 1 << 16, "c64", graph=True, profile=True)
    h = C.c_void_p()
    assert lib.atsfft_plan(C.byref(h), C.byref(d)) == A.EINVAL


def test_null_arguments():
    lib = A.load()
    assert lib.atsfft_plan(None, None) == A.EINVAL
    assert lib.atsfft_workspace_size(None, 1, None) == A.EINVAL
    assert lib.atsfft_execute(None, None, None, None, None, None, None, None, 0, None) == A.EINVAL
    assert lib.atsfft_backward(None, 1, None, None, None, None) == A.EINVAL
    assert lib.atsfft_destroy(None) == A.SUCCESS


def test_plan_without_device_reports_enodevice():
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    lib = A.load()
    d = A.default_desc(1, 1 << 16, "c64")
    h = C.c_void_p()
    assert lib.atsfft_plan(C.byref(h), C.byref(d)) == A.ENODEVICE
