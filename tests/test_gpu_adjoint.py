"""Adjoint (transpose) solves and the autograd path.  The adjoint is the
Euclidean transpose of f -> u on grid samples; the oracle's adjoint is pinned
to the dense transpose on the CPU."""
import numpy as np
import pytest
import torch

import oracle as O
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1510_08094_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.library()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("n,m", [(8, 8), (64, 64), (40, 21), (150, 75), (1024, 1024), (2048, 512)])
def test_mixed_adjoint_matches_oracle(P, n, m):
    g = np.random.default_rng(n * 3 + m).standard_normal((m, n))
    plan = P.SpherePoisson(n, m, "mixed")
    fb = host(plan.adjoint(gpu(g)))
    plan.close()
    assert rel2(fb, O.adjoint_reduced(g)) <= 1e-10


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_adjoint_dot_product(P, precision, tol):
    n, m = 512, 384
    rng = np.random.default_rng(9)
    f, g = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    plan = P.SpherePoisson(n, m, precision)
    u = host(plan.solve(gpu(f)))
    fb = host(plan.adjoint(gpu(g)))
    plan.close()
    a, b = np.vdot(u, g), np.vdot(f, fb)
    assert abs(a - b) <= tol * abs(a)


def test_autograd_gradcheck(P):
    n, m = 8, 6
    plan = P.SpherePoisson(n, m, "fp64")
    f = torch.randn(m, n, dtype=torch.float64, device="cuda", requires_grad=True)
    assert torch.autograd.gradcheck(lambda x: P.SpherePoissonFunction.apply(x, plan), (f,), eps=1e-6, atol=1e-9)
    plan.close()


def _c4_problem(r, n=2048, m=2048, L=512):
    f = S.sphere_field(4, r, n, m, L, tag=S.TAG_F)
    u_obs = S.sphere_field(4, r, n, m, L, tag=S.TAG_OBS) + S.noise(4, r, (m, n), 1e-3)
    v = S.direction(4, r, (m, n))
    return f, u_obs, v


@pytest.mark.parametrize("precision,tol_grad,tol_fd", [("fp64", 1e-11, 1e-9), ("mixed", 1e-9, 1e-8)])
def test_c4_gradient(P, precision, tol_grad, tol_fd):
    """16 right-hand sides at 2048 x 2048: loss = sum_r ||u(f_r) - u_obs_r||^2,
    gradient through SpherePoissonFunction (hand-written adjoint) against the
    oracle gradient 2 S^T (S f - u_obs) and a central difference along a seeded
    direction (exact up to rounding for a quadratic loss, step 0.1 ||f||)."""
    n = m = 2048
    R = 16
    plan = P.SpherePoisson(n, m, precision)
    worst_grad = 0.0
    worst_fd = 0.0
    for r in range(R):
        f, u_obs, v = _c4_problem(r)
        fg = gpu(f).requires_grad_(True)
        uo = gpu(u_obs)
        loss = ((P.SpherePoissonFunction.apply(fg, plan) - uo) ** 2).sum()
        loss.backward()
        grad = host(fg.grad)
        if r < 4:   # the CPU oracle on a subset keeps the test within seconds
            ref = 2.0 * O.adjoint_reduced(O.solve_reduced(f) - u_obs)
            worst_grad = max(worst_grad, rel2(grad, ref))
        h = 0.1 * np.linalg.norm(f) / np.linalg.norm(v)
        with torch.no_grad():
            jp = float(((plan.solve(gpu(f + h * v)) - uo) ** 2).sum())
            jm = float(((plan.solve(gpu(f - h * v)) - uo) ** 2).sum())
        fd = (jp - jm) / (2 * h)
        worst_fd = max(worst_fd, abs(fd - float(np.vdot(grad, v))) / abs(fd))
    plan.close()
    print("c4", precision, "grad vs oracle", worst_grad, "fd", worst_fd, flush=True)
    assert worst_grad <= tol_grad
    assert worst_fd <= tol_fd
