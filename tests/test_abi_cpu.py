"""The C-ABI library loads without a GPU, exports every symbol the header
declares, and rejects bad arguments before any device call."""
import ctypes
import os

import pytest

import paper_1510_08094_amd as P


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(P.LIB_PATH):
        from paper_1510_08094_amd import build
        build.build()
    return P.library()


def test_exports_every_header_symbol(lib):
    names = P.exported_symbols()
    assert len(names) >= 8
    for name in names:
        assert hasattr(lib, name), name


def _desc(n, m, prec=0, refine=1, tol=0.0, flags=0):
    return P.SpDesc(n, m, prec, refine, tol, flags)


@pytest.mark.parametrize("n,m,code", [
    (63, 64, 1),        # odd n: lambda + pi is not on the grid
    (2, 64, 1),         # too small
    (64, 3, 1),
    (2 * 37, 64, 2),    # prime factor 37 in n/2
    (64, 41, 2),        # prime factor 41 in m
])
def test_plan_rejects_bad_sizes(lib, n, m, code):
    pl = ctypes.c_void_p()
    d = _desc(n, m)
    assert lib.sphere_poisson_plan(ctypes.byref(pl), ctypes.byref(d), None) == code
    assert not pl.value


def test_plan_rejects_bad_desc(lib):
    pl = ctypes.c_void_p()
    assert lib.sphere_poisson_plan(ctypes.byref(pl), None, None) == 1
    assert lib.sphere_poisson_plan(None, ctypes.byref(_desc(64, 64)), None) == 1
    assert lib.sphere_poisson_plan(ctypes.byref(pl), ctypes.byref(_desc(64, 64, prec=7)), None) == 1
    assert lib.sphere_poisson_plan(ctypes.byref(pl), ctypes.byref(_desc(64, 64, refine=-1)), None) == 1
    assert lib.sphere_poisson_plan(ctypes.byref(pl), ctypes.byref(_desc(64, 64, flags=0x80)), None) == 1


def test_null_plan_calls(lib):
    assert lib.sphere_poisson_solve(None, None, None, 0.0, None, None) == 8
    assert lib.sphere_poisson_solve_adjoint(None, None, None, None, None) == 8
    assert lib.sphere_poisson_destroy(None) == 8
    assert lib.sphere_poisson_transform_roundtrip(None, None, None, None) == 8
    # a pointer that was never a plan is rejected without being dereferenced
    bogus = ctypes.c_void_p(0x1234)
    assert lib.sphere_poisson_solve(bogus, None, None, 0.0, None, None) == 8


def test_batch_argument_validation(lib):
    assert lib.sphere_poisson_solve_batch(0, None, None, None, None, 0, None, None) == 1


def test_workspace_bytes_scale(lib):
    small = lib.sphere_poisson_workspace_bytes(ctypes.byref(_desc(64, 64)))
    big = lib.sphere_poisson_workspace_bytes(ctypes.byref(_desc(1024, 1024)))
    assert 0 < small < big
    # two float64 spectra ((n/2+1) x m complex each: the theta input in runs for
    # the theta pass, its output in runs for the lambda pass), about 16 bytes
    # per sample, plus small tables
    assert 16 * 1024 * 1024 <= big < 20 * 1024 * 1024
    assert lib.sphere_poisson_workspace_bytes(ctypes.byref(_desc(63, 64))) == 0


def test_strerror(lib):
    for c in range(0, 9):
        assert len(lib.sphere_poisson_strerror(c)) > 3
    assert b"unknown" in lib.sphere_poisson_strerror(99)


def test_binding_requires_library(monkeypatch, tmp_path):
    monkeypatch.setattr(P, "_lib", None)
    monkeypatch.setattr(P, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(P.LibraryMissing):
        P.library()
