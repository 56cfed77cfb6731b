"""The C-ABI library loads and exports every function include/helm.h declares
(no compute: these run without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "helm.h")
LIB = os.path.join(ROOT, "paper_2301_10762_amd", "libhelm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(helm_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("helm_factor", "helm_solve", "helm_adjoint_solve", "helm_misfit_grad", "helm_gn_hvp",
                     "helm_factor_destroy", "helm_factor_bytes", "helm_last_error", "helm_hess_create",
                     "helm_hess_create_at", "helm_hess_apply", "helm_hess_pcg", "helm_hess_pcg_batch",
                     "helm_hess_destroy", "helm_gamma_solve", "helm_upper_grad", "helm_restrict",
                     "helm_point_sources", "helm_fwi"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_host_side_argument_checks_without_gpu():
    """Entry points reject bad grids before touching the device."""
    from paper_2301_10762_amd import helm
    L = helm.lib()
    g = helm._Grid(1, 5, 0.1, 0.1)
    out = ctypes.c_size_t(0)
    assert L.helm_factor_bytes(ctypes.byref(g), 0, ctypes.byref(out)) == helm.EINVAL
    assert b"nx >= 2" in L.helm_last_error()
    g = helm._Grid(401, 401, 0.025, 0.025)
    assert L.helm_factor_bytes(ctypes.byref(g), 0, ctypes.byref(out)) == 0
    # 401 -> 416 padded block, 401 blocks of complex128, plus the model copy
    assert out.value == 416 * 416 * 401 * 16 + 401 * 401 * 8
    assert L.helm_factor_bytes(ctypes.byref(g), 1, ctypes.byref(out)) == 0
    assert out.value == 416 * 416 * 401 * 8 + 401 * 401 * 8
    assert L.helm_factor_bytes(ctypes.byref(g), 7, ctypes.byref(out)) == helm.EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_hessian_entry_points_check_arguments_without_gpu():
    """The Hessian and preconditioner entry points reject bad arguments
    before touching the device."""
    from paper_2301_10762_amd import helm
    L = helm.lib()
    fake = ctypes.c_void_p(16)
    g = helm._Grid(9, 9, 0.1, 0.1)
    # Gamma(alpha, 0) is singular; negative alpha is not a regulariser
    assert L.helm_gamma_solve(ctypes.byref(g), 1.0, 0.0, 1, fake, fake, None) == helm.EINVAL
    assert L.helm_gamma_solve(ctypes.byref(g), -1.0, 1.0, 1, fake, fake, None) == helm.EINVAL
    assert L.helm_gamma_solve(ctypes.byref(g), 1.0, 1.0, 0, fake, fake, None) == helm.EINVAL
    bad = helm._Grid(1, 9, 0.1, 0.1)
    assert L.helm_gamma_solve(ctypes.byref(bad), 1.0, 1.0, 1, fake, fake, None) == helm.EINVAL
    # NULL context
    info = helm._Info()
    assert L.helm_hess_apply(None, 1, fake, fake, None, ctypes.byref(info)) == helm.EINVAL
    it, rr = ctypes.c_int32(0), ctypes.c_double(0)
    assert L.helm_hess_pcg(None, fake, fake, 0.0, 0.0, 1e-6, 10, None, ctypes.byref(it), ctypes.byref(rr),
                           ctypes.byref(info)) == helm.EINVAL
    # phi / grad without data, and no output handle
    w = (ctypes.c_double * 1)(1.0)
    src = (ctypes.c_int32 * 1)(40)
    rec = (ctypes.c_int32 * 1)(0)
    phi = ctypes.c_double(0)
    out = ctypes.c_void_p()
    assert L.helm_hess_create(ctypes.byref(g), fake, 1, w, None, 1, src, 1, rec, 0.0, 0.0, 0, 0.0, None,
                              ctypes.byref(phi), None, ctypes.byref(info), ctypes.byref(out)) == helm.EINVAL
    assert L.helm_hess_create(ctypes.byref(g), fake, 1, w, None, 1, src, 1, rec, 0.0, 0.0, 0, 0.0, None,
                              None, None, ctypes.byref(info), None) == helm.EINVAL
    # node indices out of range
    src_bad = (ctypes.c_int32 * 1)(81)
    assert L.helm_hess_create(ctypes.byref(g), fake, 1, w, None, 1, src_bad, 1, rec, 0.0, 0.0, 0, 0.0, None,
                              None, None, ctypes.byref(info), ctypes.byref(out)) == helm.EINVAL
    assert not out.value
    helm.lib().helm_hess_destroy(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhelm.so not built")
def test_fwi_checks_arguments_without_gpu():
    from paper_2301_10762_amd import helm
    L = helm.lib()
    fake = ctypes.c_void_p(16)
    g = helm._Grid(9, 9, 0.1, 0.1)
    w = (ctypes.c_double * 1)(1.0)
    src = (ctypes.c_int32 * 1)(40)
    rec = (ctypes.c_int32 * 1)(0)
    xz = (ctypes.c_double * 2)(0.15, 0.05)
    info = helm._FwiInfo()
    good = helm._LbfgsOpts(5, 10, 20, 1e-6, 1e-4, 0.9, 0.01)
    bad = helm._LbfgsOpts(5, 10, 20, 1e-6, 0.5, 0.4, 0.01)
    # both or neither receiver form
    sxz = (ctypes.c_double * 2)(0.35, 0.45)
    assert L.helm_fwi(ctypes.byref(g), fake, 1, w, fake, 1, src, None, 1, rec, xz, 0.0, 0.0, 0, 0.0,
                      ctypes.byref(good), None, None, ctypes.byref(info)) == helm.EINVAL
    assert L.helm_fwi(ctypes.byref(g), fake, 1, w, fake, 1, src, None, 1, None, None, 0.0, 0.0, 0, 0.0,
                      ctypes.byref(good), None, None, ctypes.byref(info)) == helm.EINVAL
    # both or neither source form
    assert L.helm_fwi(ctypes.byref(g), fake, 1, w, fake, 1, src, sxz, 1, rec, None, 0.0, 0.0, 0, 0.0,
                      ctypes.byref(good), None, None, ctypes.byref(info)) == helm.EINVAL
    # c1 >= c2
    assert L.helm_fwi(ctypes.byref(g), fake, 1, w, fake, 1, src, None, 1, rec, None, 0.0, 0.0, 0, 0.0,
                      ctypes.byref(bad), None, None, ctypes.byref(info)) == helm.EINVAL
    # a point source outside the domain
    far = (ctypes.c_double * 2)(0.35, 4.5)
    B = ctypes.c_void_p(16)
    assert L.helm_point_sources(ctypes.byref(g), 1, far, B, 81, None) == helm.EINVAL
