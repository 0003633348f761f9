"""The C-ABI library loads and exports every entry point include/tm.h declares;
argument validation runs (and fails cleanly) without a device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "tm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tm_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def L():
    from paper_1311_4462_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtm.so not built (run __graft_entry__.build())")
    return _lib.lib()


def test_every_declared_symbol_is_exported(L):
    from paper_1311_4462_amd import _lib
    names = _declared()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.EXPORTED)


def test_error_strings(L):
    for code in (0, 1, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        s = L.tm_error_string(code)
        assert s and s != b"unknown error"


def test_validation_without_device(L):
    from paper_1311_4462_amd._lib import tm_params
    h = ctypes.c_void_p()
    assert L.tm_ctx_create(ctypes.byref(h), None) == 0
    p = tm_params()
    for i, d in enumerate((4, 4, 4, 4)):
        p.dims[i] = d
    p.kappa, p.mu, p.epsilon, p.flavor, p.t_antiperiodic = 0.16, 0.1, 0.0, 1, 1
    # sizes: FP64 one flavour = 192 B per site, FP16 = 48 B + 4 B scale (256-B rounded)
    assert L.tm_spinor_bytes(ctypes.byref(p), 0, 1) == 128 * 192
    assert L.tm_spinor_bytes(ctypes.byref(p), 1, 2) == 2 * 128 * 96
    assert L.tm_spinor_bytes(ctypes.byref(p), 2, 1) == 128 * 48 + 512
    g = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)
    p.dims[2] = 5
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 3) == -2
    assert b"not even" in L.tm_last_error(h)
    assert L.tm_spinor_bytes(ctypes.byref(p), 0, 1) == 0
    p.dims[2] = 4
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 16, 3) == -1   # recon
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 0) == -4   # precision
    p.flavor = 7
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 3) == -1
    # singular doublet twist: 1 + a^2 - b^2 = 0 with a = 2 k mu, b = 2 k eps
    p.flavor, p.kappa, p.mu, p.epsilon = 2, 0.25, 1.0, 5 ** 0.5
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 3) == -5
    p.epsilon = float("nan")
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 3) == -1
    assert L.tm_mat_pc(h, dummy, dummy, None, 0, 0, 0, 1) == -1
    assert L.tm_cg(h, dummy, dummy, None, None, None) == -1
    # the largest lattice: 2e8 sites per parity (site indices stay 32-bit)
    p.flavor, p.kappa, p.mu, p.epsilon = 1, 0.16, 0.1, 0.0
    for i, d in enumerate((1024, 1024, 512, 2)):
        p.dims[i] = d
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 3) == -9
    assert b"too large" in L.tm_last_error(h)
    assert L.tm_spinor_bytes(ctypes.byref(p), 0, 1) == 0
    assert L.tm_ctx_destroy(h) == 0


def test_validation_of_newer_entry_points_without_device(L):
    """Twisted-clover parameters, 8-real links, full-system solves and the
    spin basis of pack/unpack are validated before any device work."""
    from paper_1311_4462_amd._lib import tm_cg_result, tm_params, tm_solve_params
    h = ctypes.c_void_p()
    assert L.tm_ctx_create(ctypes.byref(h), None) == 0
    p = tm_params()
    for i, d in enumerate((4, 4, 4, 4)):
        p.dims[i] = d
    p.kappa, p.mu, p.epsilon, p.flavor, p.t_antiperiodic = 0.16, 0.1, 0.0, 1, 1
    g = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)
    # recon 8 is accepted as a value; 10 is not
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 10, 3) == -1
    # twisted clover: FP64 / FP32 only, not with 8-real links, finite c_sw
    p.csw = 1.5
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 1 << 2) == -4
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 8, 3) == -1
    p.csw = float("inf")
    assert L.tm_gauge_create(h, ctypes.byref(g), dummy, ctypes.byref(p), 12, 3) == -1
    p.csw = 0.0
    # spin basis
    assert L.tm_spinor_pack(h, dummy, dummy, ctypes.byref(p), 0, 0, 1, 2) == -1
    assert L.tm_spinor_unpack(h, dummy, dummy, ctypes.byref(p), 0, 0, 1, -1) == -1
    # full-system solve: parameter checks come first
    sp = tm_solve_params()
    res = (tm_cg_result * 1)()
    assert L.tm_solve(h, dummy, dummy, dummy, dummy, None, None, res) == -1
    sp.cg.tol, sp.cg.maxiter, sp.cg.nrhs = 1e-10, 10, 1
    assert L.tm_solve(h, dummy, dummy, dummy, dummy, None, ctypes.byref(sp), res) == -1   # null gauge
    assert L.tm_ctx_destroy(h) == 0
