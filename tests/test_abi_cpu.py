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


def _batch(lib, sizes, fptrs, uptrs, prec=1, refine=1, flags=0):
    k = len(sizes)
    ns = (ctypes.c_int * k)(*[s[0] for s in sizes])
    ms = (ctypes.c_int * k)(*[s[1] for s in sizes])
    fp = (ctypes.c_void_p * k)(*fptrs)
    up = (ctypes.c_void_p * k)(*uptrs)
    out = ctypes.c_void_p()
    d = _desc(0, 0, prec, refine, 0.0, flags)
    code = lib.sphere_poisson_batch_plan(ctypes.byref(out), k, ns, ms, fp, up, ctypes.byref(d), None)
    assert not out.value
    return code


def test_batch_argument_validation(lib):
    """The batch plan validates before any device call; the pointers below
    are never dereferenced."""
    out = ctypes.c_void_p()
    d = _desc(0, 0, 1)
    assert lib.sphere_poisson_batch_plan(ctypes.byref(out), 0, None, None, None, None, ctypes.byref(d), None) == 1
    assert lib.sphere_poisson_batch_plan(None, 1, None, None, None, None, ctypes.byref(d), None) == 1
    MB = 1 << 20
    a, b, c = 0x10000000, 0x20000000, 0x30000000
    assert _batch(lib, [(64, 64)], [a], [b], prec=3) == 1                      # precision
    assert _batch(lib, [(64, 64)], [a], [b], refine=0) == 1                    # mixed needs a correction
    assert _batch(lib, [(64, 64)], [a], [b], refine=5) == 1                    # at most four
    assert _batch(lib, [(64, 64)], [a], [b], flags=0x80) == 1                  # unknown flag
    assert _batch(lib, [(63, 64)], [a], [b]) == 1                              # odd n
    assert _batch(lib, [(64, 64)], [None], [b]) == 1                           # null pointer
    # aliasing: a u over its own f, over another problem's f or u; shared f buffers are fine
    assert _batch(lib, [(64, 64)], [a], [a + 8]) == 6
    assert _batch(lib, [(64, 64), (64, 64)], [a, b], [c, a + 4096]) == 6       # u1 inside f0
    assert _batch(lib, [(64, 64), (64, 64)], [a, b], [c, c + 8]) == 6          # u0 and u1 overlap
    assert _batch(lib, [(64, 64), (128, 64)], [a, c + 64 * 1024 - 8], [c + MB, c]) == 6   # f1 overlaps u1's end
    assert lib.sphere_poisson_solve_batch(None, None, None) == 8
    assert lib.sphere_poisson_solve_batch(ctypes.c_void_p(0x1234), None, None) == 8
    assert lib.sphere_poisson_batch_destroy(None) == 8
    assert lib.sphere_poisson_get_info(None, None, None) == 8


def test_batch_alias_rule_on_disjoint_buffers(lib):
    """Disjoint outputs and shared inputs pass the alias check: the plan then
    proceeds to the device and fails there without a GPU (no device), not with
    SP_ERR_ALIAS."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("with a GPU the plan would be built on these never-launched fake pointers")
    a, c = 0x10000000, 0x30000000
    code = _batch(lib, [(64, 64), (64, 64)], [a, a], [c, c + 64 * 64 * 8])
    assert code not in (1, 6)


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


def test_widened_calls_reject_null_plan(lib):
    """The calculus, integration, low-rank and evaluation calls check the plan
    before anything else."""
    assert lib.sphere_poisson_tangential_gradient(None, None, None, None, None, None) == 8
    assert lib.sphere_poisson_integral(None, None, None, None) == 8
    assert lib.sphere_poisson_solve_lowrank(None, 3, None, None, None, None, 0.0, None, None) == 8
    assert lib.sphere_poisson_eval_lowrank(None, 3, None, None, None, 10, None, None, None) == 8


def test_ge_argument_validation(lib):
    """The Gaussian-elimination constructor validates sizes, parameters,
    pointers, workspace and aliasing before any device call (the pointers
    below are never dereferenced)."""
    n, m = 16, 12
    wb = lib.sphere_poisson_ge_workspace_bytes(n, m)
    assert wb >= n * m * 8
    assert lib.sphere_poisson_ge_workspace_bytes(15, m) == 0
    assert lib.sphere_poisson_ge_workspace_bytes(n, 0) == 0
    vp = ctypes.c_void_p
    f, work, d, c, r = 0x100000, 0x200000, 0x300000, 0x400000, 0x500000

    def call(steps=2, alpha=0.01, tol=0.0, wbytes=wb, ff=f, ww=work, dd=d, cc=c, rr=r, nn=n):
        return lib.sphere_poisson_ge_lowrank(nn, m, vp(ff), steps, alpha, tol, vp(ww), wbytes, vp(dd), vp(cc), vp(rr),
                                             None, None)

    assert call(steps=0) == 1
    assert call(alpha=1.5) == 1 and call(alpha=-1e-3) == 1
    assert call(tol=-1.0) == 1 and call(tol=float("nan")) == 1
    assert call(nn=15) == 1
    assert call(ff=None) == 1 and call(ww=None) == 1 and call(dd=None) == 1
    assert call(wbytes=wb - 1) == 1
    assert call(ww=work + 8) == 1 and call(rr=r + 8) == 1       # 16-byte alignment
    assert call(cc=f) == 6                                         # output over the input
    assert call(dd=work + 64) == 6                                 # output over the workspace
    assert call(cc=r) == 6                                         # outputs over each other
