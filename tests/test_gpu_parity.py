"""Parity of the HIP path (through the C ABI) with the CPU oracle and with
closed-form solutions.  Float64 bar: relative 2-norm error <= 1e-12."""
import numpy as np
import pytest
import torch

import oracle as O
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12


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
    return t.cpu().numpy()


def solve(P, f, integral=0.0, precision="fp64"):
    m, n = f.shape
    plan = P.SpherePoisson(n, m, precision)
    u = host(plan.solve(gpu(f), integral))
    plan.close()
    return u


def field(n, m, L, seed, with_solution=False):
    return S.sphere_field(seed, 0, n, m, L, with_solution=with_solution)


# (10000, 40) and (40, 10000): the compiled-in length-5000 transform in the
# lambda direction alone, and in the theta direction (real parts, m/2 = 5000)
# alone, each with a short ragged other direction
SIZES = [(64, 64), (4, 4), (8, 4), (40, 21), (150, 75), (96, 60), (210, 143), (68, 38), (46, 58),
         (62, 31), (128, 2048), (2048, 128), (1984, 1984), (256, 200), (10000, 40), (40, 10000)]


@pytest.mark.parametrize("n,m", SIZES)
def test_transforms_roundtrip(P, n, m):
    print("roundtrip", n, m, flush=True)
    f = np.random.default_rng(n * 7 + m).standard_normal((m, n))
    plan = P.SpherePoisson(n, m)
    out = host(plan.roundtrip(gpu(f)))
    plan.close()
    ref = f * np.sin(O.theta_grid(m))[:, None] ** 2
    assert rel2(out, ref) <= 1e-14


@pytest.mark.parametrize("n,m", SIZES)
def test_solve_matches_oracle(P, n, m):
    print("solve", n, m, flush=True)
    L = max(1, min(n // 2 - 1, m - 3, 40))
    f = field(n, m, L, 11)
    f = f + 1e-3 * np.random.default_rng(m).standard_normal(f.shape)   # not band-limited
    u = solve(P, f)
    assert rel2(u, O.solve_reduced(f)) <= TOL64


def test_c0_closed_form(P):
    """64 x 64, l <= 16: closed form and oracle."""
    f, u_exact = field(64, 64, 16, 0, with_solution=True)
    u = solve(P, f)
    assert rel2(u, u_exact) <= TOL64
    assert rel2(u, O.solve_reduced(f)) <= TOL64
    assert rel2(u, O.solve_literal(f)) <= TOL64


def test_c1_closed_form(P):
    """1024 x 1024, l <= 256."""
    f, u_exact = S.sphere_field(1, 0, 1024, 1024, 256, with_solution=True)
    u = solve(P, f)
    assert rel2(u, u_exact) <= TOL64
    assert rel2(u, O.solve_reduced(f)) <= TOL64


def test_paper_example_sin50xyz(P):
    """Section 5 example: f = sin(50 xyz), m_p = n = 150 (75 theta samples).
    No printed values: parity with the oracle only."""
    x, y, z = S.cartesian(150, 75)
    f = np.sin(50 * x * y * z)
    assert rel2(solve(P, f), O.solve_reduced(f)) <= TOL64


@pytest.mark.parametrize("c", [1.0, -2.5])
def test_integral_constraint(P, c):
    f, u_exact = field(48, 40, 10, 3, with_solution=True)
    u = solve(P, f, integral=c)
    assert np.max(np.abs(u - (u_exact + c / (4 * np.pi)))) <= 1e-13
    assert abs(O.sum2(u) - c) <= 1e-12


def test_info_reports_integral_of_f(P):
    f = field(64, 48, 12, 4) + 0.75          # non-zero mean: integral 4 pi * 0.75
    plan = P.SpherePoisson(64, 48, sync_info=True)
    u = host(plan.solve(gpu(f)))
    assert abs(plan.info.f_integral - 4 * np.pi * 0.75) <= 1e-12
    assert plan.info.status == 0
    assert rel2(u, O.solve_reduced(f)) <= TOL64
    plan.close()


@pytest.mark.parametrize("n,m", [(8, 8), (64, 64), (40, 21), (150, 75), (1024, 1024)])
def test_adjoint_matches_oracle(P, n, m):
    g = np.random.default_rng(n + m).standard_normal((m, n))
    plan = P.SpherePoisson(n, m)
    fb = host(plan.adjoint(gpu(g)))
    plan.close()
    assert rel2(fb, O.adjoint_reduced(g)) <= TOL64


def test_adjoint_dot_product(P):
    n, m = 256, 192
    rng = np.random.default_rng(5)
    f, g = rng.standard_normal((m, n)), rng.standard_normal((m, n))
    plan = P.SpherePoisson(n, m)
    u = host(plan.solve(gpu(f)))
    fb = host(plan.adjoint(gpu(g)))
    plan.close()
    a, b = np.vdot(u, g), np.vdot(f, fb)
    assert abs(a - b) <= 1e-12 * abs(a)


def test_repeat_is_bitwise_deterministic(P):
    f = field(512, 384, 60, 6)
    plan = P.SpherePoisson(512, 384)
    a = host(plan.solve(gpu(f)))
    b = host(plan.solve(gpu(f)))
    plan.close()
    assert np.array_equal(a, b)


def test_errors(P):
    plan = P.SpherePoisson(64, 32)
    f = gpu(np.zeros((32, 64)))
    with pytest.raises(P.SpError) as e:
        plan.solve(f, out=f)
    assert e.value.code == 6
    with pytest.raises(TypeError):
        plan.solve(f.float())
    with pytest.raises(ValueError):
        plan.solve(gpu(np.zeros((64, 32))))
    plan.close()
    with pytest.raises(P.SpError) as e:
        plan._plan = plan._plan or None
        P._check(P.library().sphere_poisson_destroy(plan._plan))
    assert e.value.code == 8


def test_c2_closed_form_and_oracle(P):
    """10000 x 10000 (1e8 samples), l <= 2000, float64."""
    n = m = 10000
    print("c2 synth", flush=True)
    f, u_exact = S.sphere_field(2, 0, n, m, 2000, with_solution=True)
    print("c2 gpu", flush=True)
    u = solve(P, f)
    e_exact = rel2(u, u_exact)
    print("c2 rel err vs closed form", e_exact, flush=True)
    assert e_exact <= TOL64
    del u_exact
    print("c2 oracle", flush=True)
    assert rel2(u, O.solve_reduced(f)) <= TOL64
