"""Pointwise evaluation of a low-rank function on the GPU (Section 4, Pointwise
evaluation), through the C ABI: parity with the oracle's explicit sums, the
interpolation property at the grid nodes, polynomials anywhere (points off
the sphere are projected), band-limited fields at the nodes of another grid.
Bar: relative 2-norm error <= 1e-12 (the Horner sums and the oracle's
matrix products differ only in rounding, about m eps times the size of the
coefficients)."""
import ctypes

import numpy as np
import pytest
import torch

import oracle.evaluate as OE
import oracle.lowrank as OL
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def P():
    import paper_1510_08094_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.library()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def points(count, seed, radius=1.0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, 3))
    return v * (radius / np.linalg.norm(v, axis=1))[:, None]


def evaluate(P, n, m, d, C, R, pts):
    plan = P.SpherePoisson(n, m, "fp64")
    try:
        out = plan.eval_lowrank(gpu(d), gpu(C), gpu(R), gpu(pts))
        torch.cuda.synchronize()
        return out.cpu().numpy()
    finally:
        plan.close()


# (n, m, K, L): N = n/2 even and odd, m below and above the unroll, ragged point counts
CASES = [(16, 12, 3, 5), (40, 21, 9, 8), (42, 31, 7, 12), (64, 33, 5, 15), (150, 150, 25, 40), (8, 4, 3, 1)]


@pytest.mark.parametrize("n,m,K,L", CASES)
def test_matches_oracle(P, n, m, K, L):
    print("eval", n, m, K, L, flush=True)
    d, C, R = S.lowrank_factors(31, K, n, m, K, L)
    pts = points(777, n + m, radius=1.3)
    got = evaluate(P, n, m, d, C, R, pts)
    ref = OE.evaluate_lowrank(d, C, R, pts[:, 0], pts[:, 1], pts[:, 2])
    assert rel2(got, ref) <= TOL


@pytest.mark.parametrize("n,m,K", [(16, 12, 4), (42, 31, 6), (150, 150, 20)])
def test_reproduces_samples_at_nodes(P, n, m, K):
    rng = np.random.default_rng(n * m)
    d, C, R = rng.standard_normal(K), rng.standard_normal((K, m)), rng.standard_normal((K, n))
    x, y, z = S.cartesian(n, m)
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    got = evaluate(P, n, m, d, C, R, pts).reshape(m, n)
    assert rel2(got, OL.lowrank_grid(d, C, R)) <= TOL


def _poly_factors(m, n):
    th = (np.arange(m) + 0.5) * np.pi / m
    lam = -np.pi + 2 * np.pi * np.arange(n) / n
    C = np.vstack([np.sin(th) ** 2 * np.cos(th), np.cos(th), np.sin(th) ** 2, np.sin(th)])
    R = np.vstack([0.5 * np.sin(2 * lam), np.ones(n), np.cos(lam) ** 2, np.sin(lam)])
    return np.array([1.0, 1.0, 1.0, -1.0]), C, R


@pytest.mark.parametrize("n,m", [(16, 12), (150, 150)])
def test_polynomial_closed_form(P, n, m):
    """x y z + z + x^2 - y at random points of radius 1 and 2.5, the poles and
    the lambda = +-pi seam."""
    d, C, R = _poly_factors(m, n)
    pts = np.vstack([points(500, 7, 1.0), points(500, 8, 2.5),
                     [[0, 0, 1], [0, 0, -1], [-1, 0, 0], [-1, -0.0, 0.3]]])
    got = evaluate(P, n, m, d, C, R, pts)
    rho = np.linalg.norm(pts, axis=1)
    x, y, z = (pts / rho[:, None]).T
    assert np.max(np.abs(got - (x * y * z + z + x * x - y))) <= 1e-13


@pytest.mark.parametrize("L,n,m,n2,m2", [(12, 64, 48, 100, 75), (20, 150, 150, 64, 33)])
def test_band_limited_field_on_another_grid(P, L, n, m, n2, m2):
    d, C, R = S.sphere_field_factors(8, L, n, m, L)
    x, y, z = S.cartesian(n2, m2)
    pts = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    got = evaluate(P, n, m, d, C, R, pts).reshape(m2, n2)
    assert rel2(got, S.sphere_field(8, L, n2, m2, L)) <= TOL


def test_million_points_sampled(P):
    """10^6 points of a rank-25 field on 150 x 150; 3000 of them against the oracle."""
    n = m = 150
    d, C, R = S.sphere_field_factors(9, 0, n, m, 12)
    pts = points(10 ** 6, 10)
    got = evaluate(P, n, m, d, C, R, pts)
    idx = np.random.default_rng(11).choice(10 ** 6, 3000, replace=False)
    ref = OE.evaluate_lowrank(d, C, R, pts[idx, 0], pts[idx, 1], pts[idx, 2])
    assert rel2(got[idx], ref) <= TOL


def test_errors_and_empty(P):
    n, m = 16, 12
    lib = P.library()
    plan = P.SpherePoisson(n, m, "fp64")
    d, C, R = S.lowrank_factors(32, 0, n, m, m, 3)
    dg, Cg, Rg = gpu(d), gpu(C), gpu(R)
    pts = gpu(points(10, 1))
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    vp = ctypes.c_void_p

    def call(rank, cnt, xyz, o):
        return lib.sphere_poisson_eval_lowrank(plan._plan, rank, vp(dg.data_ptr()), vp(Cg.data_ptr()),
                                               vp(Rg.data_ptr()), cnt, vp(xyz), vp(o), None)

    assert call(3, 0, None, None) == 0
    assert call(3, -1, pts.data_ptr(), out.data_ptr()) == 1
    assert call(0, 10, pts.data_ptr(), out.data_ptr()) == 1
    assert call(n // 2 + 2, 10, pts.data_ptr(), out.data_ptr()) == 1
    assert call(3, 10, None, out.data_ptr()) == 1
    assert call(3, 10, pts.data_ptr(), pts.data_ptr() + 8) == 6
    assert call(n // 2 + 1, 10, pts.data_ptr(), out.data_ptr()) == 0
    torch.cuda.synchronize()
    plan.close()
