"""The C-ABI library builds for gfx950, loads, exports every declared entry
point and rejects invalid arguments on the host, before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mecdf.h")
LIB = os.path.join(ROOT, "paper_2005_03246_amd", "_lib", "libmecdf.so")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?(?:int|void|char)\s*\*?\s*(\w+)\s*\(", src, re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2005_03246_amd import build

        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_paper_entry_points():
    names = declared_functions()
    for n in ["ecdf_grid", "esf_grid", "ecdf_points", "esf_points",
              "kde_laplace", "kreg_laplace"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for n in declared_functions():
        assert hasattr(lib, n), n


def _c(lib, name, argtypes):
    f = getattr(lib, name)
    f.argtypes = argtypes
    f.restype = ctypes.c_int
    return f


P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64


def test_host_validation_errors(lib):
    lib.mecdf_last_error.restype = ctypes.c_char_p
    grid = _c(lib, "ecdf_grid", [I, I64, P, P, P, P, P, I, P])
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    M = (ctypes.c_int64 * 2)(3, 3)
    z_ok = (ctypes.c_double * 6)(0, 1, 2, 0, 1, 2)
    z_bad = (ctypes.c_double * 6)(0, 2, 1, 0, 1, 2)
    z_nan = (ctypes.c_double * 6)(0, float("nan"), 2, 0, 1, 2)
    assert grid(0, 10, fake, None, M, z_ok, fake, 0, None) == -1
    assert grid(7, 10, fake, None, M, z_ok, fake, 0, None) == -1
    assert grid(2, -1, fake, None, M, z_ok, fake, 0, None) == -1
    assert grid(2, 10, None, None, M, z_ok, fake, 0, None) == -1
    assert grid(2, 10, fake, None, M, z_bad, fake, 0, None) == -1
    assert b"strictly increasing" in lib.mecdf_last_error()
    assert grid(2, 10, fake, None, M, z_nan, fake, 0, None) == -1
    assert grid(2, 10, fake, None, None, z_ok, fake, 0, None) == -1
    assert grid(2, 10, fake, None, M, z_ok, None, 0, None) == -1
    assert grid(2, 10, fake, None, M, z_ok, fake, 5, None) == -1
    assert grid(2, 0, fake, fake, M, z_ok, fake, 0, None) == -1  # weighted N=0
    M0 = (ctypes.c_int64 * 2)(0, 3)
    assert grid(2, 10, fake, None, M0, z_ok, fake, 0, None) == -1
    big = (ctypes.c_int64 * 1)(5000)
    zb = (ctypes.c_double * 5000)(*range(5000))
    assert grid(1, 10, fake, None, big, zb, fake, 0, None) == -4
    pts = _c(lib, "ecdf_points", [I, I64, P, P, P, I, P])
    assert pts(0, 10, fake, None, fake, 0, None) == -1
    assert pts(2, 10, fake, None, None, 0, None) == -1
    assert pts(2, 1 << 31, fake, None, fake, 0, None) == -4
    kde = _c(lib, "kde_laplace", [I, I64, P, P, I, P, P, P, I, P])
    h = (ctypes.c_double * 2)(0.1, 0.1)
    hneg = (ctypes.c_double * 2)(0.1, -0.1)
    assert kde(2, 1, fake, None, 1, h, fake, None, 0, None) == -1   # N < 2
    assert kde(7, 10, fake, None, 1, h, fake, None, 0, None) == -1  # d > 6
    h4 = (ctypes.c_double * 4)(0.1, 0.1, 0.1, 0.1)
    assert kde(4, (1 << 20) + 1, fake, None, 1, h4, fake, None, 0, None) == -4  # direct sums
    assert kde(3, (1 << 24) + 1, fake, None, 1, h4, fake, None, 0, None) == -4
    assert kde(2, 10, fake, None, 0, h, fake, None, 0, None) == -1
    assert kde(2, 10, fake, None, 1, hneg, fake, None, 0, None) == -1
    assert kde(2, 10, fake, None, 1, h, None, None, 0, None) == -1
    kreg = _c(lib, "kreg_laplace", [I, I64, P, P, I, P, P, P, I, P])
    assert kreg(2, 10, fake, None, 1, h, fake, None, 0, None) == -1  # y NULL
    train = _c(lib, "mecdf_bw_train", [I, P, P, I, P, I, ctypes.c_float, ctypes.c_float,
                                       ctypes.c_uint64, P, P, P, ctypes.c_char_p, P, P])
    hg = (ctypes.c_double * 3)(0.1, 0.2, 0.4)
    hg_bad = (ctypes.c_double * 3)(0.1, 0.4, 0.2)
    st = ctypes.c_int64(0)
    ref = ctypes.byref(st)
    assert train(0, fake, fake, 3, hg, 10, 1e-3, 0.0, 1, fake, fake, None, None, ref, None) == -1
    assert train(4, fake, fake, 3, hg, 10, 0.0, 0.0, 1, fake, fake, None, None, ref, None) == -1
    assert train(4, fake, fake, 3, hg, 10, 1e-3, -1.0, 1, fake, fake, None, None, ref, None) == -1
    assert train(4, fake, fake, 3, hg_bad, 10, 1e-3, 0.0, 1, fake, fake, None, None, ref,
                 None) == -1
    assert train(4, fake, None, 3, hg, 10, 1e-3, 0.0, 1, fake, fake, None, None, ref, None) == -1
    assert train(4, fake, fake, 3, hg, 10, 1e-3, 0.0, 1, fake, fake, None, None, None, None) == -1
    batched = _c(lib, "mecdf_kde_lcv_batched", [P, I, P, P, P, P, I, P])
    assert batched(None, 0, None, None, fake, None, 0, None) == -1
    lib.mecdf_strerror.restype = ctypes.c_char_p
    assert lib.mecdf_strerror(-1) == b"invalid argument"
    assert lib.mecdf_strerror(-5) == b"file input/output error"


def test_grid_kernel_sum_validation(lib):
    fake = ctypes.c_void_p(0x1000)
    M = (ctypes.c_int64 * 5)(3, 3, 3, 3, 3)
    z = (ctypes.c_double * 15)(*([0.0, 1.0, 2.0] * 5))
    h = (ctypes.c_double * 5)(0.1, 0.1, 0.1, 0.1, 0.1)
    hneg = (ctypes.c_double * 5)(0.1, -0.1, 0.1, 0.1, 0.1)
    for name in ("kde_laplace_grid", "kde_matern32_grid", "kreg_laplace_grid",
                 "kreg_matern32_grid"):
        f = _c(lib, name, [I, I64, P, P, P, P, I, P, P, I, P])
        reg = name.startswith("kreg")
        w = fake if reg else None
        assert f(2, 0, fake, w, M, z, 1, h, fake, 0, None) == -1       # N < 1
        assert f(2, 10, fake, w, M, z, 0, h, fake, 0, None) == -1      # nh < 1
        assert f(2, 10, fake, w, M, z, 1, hneg, fake, 0, None) == -1   # h <= 0
        assert f(2, 10, fake, w, M, z, 1, h, None, 0, None) == -1      # no output
        if reg:
            assert f(2, 10, fake, None, M, z, 1, h, fake, 0, None) == -1  # y NULL
    # d beyond 6 is refused before anything is read or launched
    mk = _c(lib, "kde_matern32_grid", [I, I64, P, P, P, P, I, P, P, I, P])
    assert mk(7, 10, fake, None, M, z, 1, h, fake, 0, None) == -1


def test_arbitrary_point_queries_validation(lib):
    fake = ctypes.c_void_p(0x1000)
    ed = _c(lib, "ecdf_delta_at", [I, I64, P, P, I64, P, P, P, I, P])
    assert ed(2, 0, fake, None, 5, fake, None, fake, 0, None) == -1     # N < 1
    assert ed(2, 10, fake, None, -1, fake, None, fake, 0, None) == -1   # Q < 0
    assert ed(2, 10, fake, None, 5, None, None, fake, 0, None) == -1    # z NULL
    assert ed(2, 10, fake, None, 5, fake, None, None, 0, None) == -1    # F NULL
    assert ed(2, 10, fake, None, 0, None, None, None, 0, None) == 0     # nothing to do
    assert ed(2, 10, fake, None, (1 << 26) + 1, fake, None, fake, 0, None) == -4
    ku = _c(lib, "kde_uniform", [I, I64, P, P, I64, P, I, P, P, I, P])
    h = (ctypes.c_double * 2)(0.1, 0.2)
    hneg = (ctypes.c_double * 2)(0.1, 0.0)
    assert ku(2, 10, fake, None, 5, fake, 0, h, fake, 0, None) == -1     # nh < 1
    assert ku(2, 10, fake, None, 5, fake, 1, hneg, fake, 0, None) == -1  # h <= 0
    assert ku(2, 10, fake, None, 5, fake, 1, None, fake, 0, None) == -1
    assert ku(2, 10, fake, None, 5, fake, 1, h, None, 0, None) == -1
    assert ku(2, 10, fake, None, (1 << 24) + 1, fake, 1, h, fake, 0, None) == -4
