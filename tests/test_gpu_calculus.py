"""Tangential derivatives (Section 4, eq. diff_x/y/z) on the GPU against the
coefficient-space oracle (eq. dfdx, Msin) and against closed forms: the
surface gradient of the restriction of a polynomial F(x, y, z) is
grad F - (p . grad F) p."""
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
    return t.cpu().numpy()


def rel3(a, b):
    num = sum(np.linalg.norm(x - y) ** 2 for x, y in zip(a, b))
    den = sum(np.linalg.norm(y) ** 2 for y in b)
    return float(np.sqrt(num / den))


def tol(n, m):
    """Rounding of the float64 path: each transform leaves a floor of about
    eps |f| on every coefficient; differentiation multiplies coefficient k (or
    q) by k <= n/2 (q <= m), and the division by sin(theta) in coefficient
    space sums up to m/2 coefficients of one parity (a random walk,
    sqrt(m/2)).  Relative error: a few eps max(n/2, m) sqrt(m)."""
    eps = np.finfo(np.float64).eps
    return max(1e-12, 4 * eps * max(n // 2, m) * np.sqrt(m))


def grid_xyz(m, n):
    th = O.theta_grid(m)[:, None]
    lam = O.lambda_grid(n)[None, :]
    return np.cos(lam) * np.sin(th), np.sin(lam) * np.sin(th), np.cos(th) * np.ones_like(lam)


def gradient(P, f, precision="fp64"):
    m, n = f.shape
    plan = P.SpherePoisson(n, m, precision)
    try:
        return tuple(host(g) for g in plan.tangential_gradient(gpu(f)))
    finally:
        plan.close()


# even and odd m (one real part per theta workgroup / complex line), radices
# up to 31, ragged lambda blocks
SIZES = [(64, 64), (40, 21), (150, 75), (96, 60), (46, 58), (62, 31), (256, 200), (128, 130), (1984, 248)]


@pytest.mark.parametrize("n,m", SIZES)
def test_gradient_matches_oracle(P, n, m):
    print("gradient", n, m, flush=True)
    L = max(1, min(n // 2 - 2, m - 3, 40))
    f = S.sphere_field(41, 0, n, m, L)
    got = gradient(P, f)
    ref = O.tangential_gradient(f)
    assert rel3(got, ref) <= tol(n, m), (n, m)


_EXPS = [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c <= 4]
_COEF = np.random.default_rng(7).standard_normal(len(_EXPS))


def _quartic(x, y, z):
    return sum(c * x ** a * y ** b * z ** e for c, (a, b, e) in zip(_COEF, _EXPS))


def _quartic_grad(x, y, z):
    gx = sum(c * a * x ** max(a - 1, 0) * y ** b * z ** e for c, (a, b, e) in zip(_COEF, _EXPS) if a)
    gy = sum(c * b * x ** a * y ** max(b - 1, 0) * z ** e for c, (a, b, e) in zip(_COEF, _EXPS) if b)
    gz = sum(c * e * x ** a * y ** b * z ** max(e - 1, 0) for c, (a, b, e) in zip(_COEF, _EXPS) if e)
    return gx, gy, gz


@pytest.mark.parametrize("n,m", [(16, 12), (96, 64), (10000, 40), (40, 10000)])
def test_gradient_quartic_closed_form(P, n, m):
    """(10000, 40) and (40, 10000) run the compiled-in length-5000 transforms."""
    print("quartic", n, m, flush=True)
    x, y, z = grid_xyz(m, n)
    got = gradient(P, _quartic(x, y, z))
    ref = O.polynomial_surface_gradient(_quartic_grad, m, n)
    assert rel3(got, ref) <= tol(n, m), (n, m)


def test_gradient_paper_example(P):
    """Section 4: d^t cos(theta)/dx = -x z."""
    m, n = 32, 48
    x, y, z = grid_xyz(m, n)
    gx, gy, gz = gradient(P, z.copy())
    assert np.max(np.abs(gx + x * z)) <= 1e-13
    assert np.max(np.abs(gy + y * z)) <= 1e-13
    assert np.max(np.abs(gz - (1 - z * z))) <= 1e-13


def test_gradient_mixed_plan_is_float64(P):
    n, m = 96, 60
    f = S.sphere_field(42, 0, n, m, 20)
    assert rel3(gradient(P, f, "mixed"), O.tangential_gradient(f)) <= 1e-12


def test_gradient_c2_closed_form(P):
    """n = m = 10000 (10^8 samples): F = x y z + z^2 - 3 x^2 y, every
    component against its closed form on a sample of rows."""
    n = m = 10000
    th = torch.tensor(O.theta_grid(m), dtype=torch.float64, device="cuda")[:, None]
    lam = torch.tensor(O.lambda_grid(n), dtype=torch.float64, device="cuda")[None, :]
    x, y, z = torch.cos(lam) * torch.sin(th), torch.sin(lam) * torch.sin(th), torch.cos(th).expand(m, n)
    f = (x * y * z + z * z - 3 * x * x * y).contiguous()
    plan = P.SpherePoisson(n, m, "fp64")
    g = plan.tangential_gradient(f)
    torch.cuda.synchronize()
    rows = torch.arange(0, m, 97, device="cuda")
    xs, ys, zs = x[rows], y[rows], z[rows]
    Fx, Fy, Fz = ys * zs - 6 * xs * ys, xs * zs - 3 * xs * xs, xs * ys + 2 * zs
    rad = xs * Fx + ys * Fy + zs * Fz
    ref = (Fx - rad * xs, Fy - rad * ys, Fz - rad * zs)
    got = tuple(c[rows] for c in g)
    err = float(torch.sqrt(sum(((a - b) ** 2).sum() for a, b in zip(got, ref)) / sum((b ** 2).sum() for b in ref)))
    plan.close()
    print("c2 gradient rel err", err, flush=True)
    assert err <= tol(n, m)


def test_gradient_errors(P):
    f = gpu(np.zeros((32, 32)))
    a, b = torch.empty_like(f), torch.empty_like(f)
    plan = P.SpherePoisson(32, 32, "fp64")
    with pytest.raises(P.SpError) as e:
        plan.tangential_gradient(f, outs=(f, a, b))
    assert e.value.code == 6
    with pytest.raises(P.SpError) as e:
        plan.tangential_gradient(f, outs=(a, a, b))
    assert e.value.code == 6
    plan.close()


def tol2(n, m):
    """Two spectral differentiations in a row (e.g. vorticity of n x grad):
    the rounding floor is amplified twice by the gain of one."""
    k = max(n // 2, m) * np.sqrt(m)
    return max(1e-11, np.finfo(np.float64).eps * k * k)


def _plan_call(P, n, m, name, *args):
    plan = P.SpherePoisson(n, m, "fp64")
    try:
        res = getattr(plan, name)(*[gpu(a) for a in args])
        return tuple(host(r) for r in res) if isinstance(res, tuple) else host(res)
    finally:
        plan.close()


@pytest.mark.parametrize("n,m", [(64, 64), (40, 21), (96, 60), (128, 130)])
def test_vector_calculus_matches_oracle(P, n, m):
    print("vector calculus", n, m, flush=True)
    L = max(1, min(n // 2 - 2, m - 3, 20))
    fx, fy, fz = (S.sphere_field(61 + c, 0, n, m, L) for c in range(3))
    assert rel3(_plan_call(P, n, m, "curl_scalar", fx), O.curl_scalar(fx)) <= tol(n, m)
    assert rel2(_plan_call(P, n, m, "divergence", fx, fy, fz), O.divergence(fx, fy, fz)) <= tol(n, m)
    assert rel3(_plan_call(P, n, m, "curl", fx, fy, fz), O.curl(fx, fy, fz)) <= tol(n, m)
    assert rel2(_plan_call(P, n, m, "vorticity", fx, fy, fz), O.vorticity(fx, fy, fz)) <= tol(n, m)


@pytest.mark.parametrize("n,m", [(256, 200), (1024, 512)])
def test_laplacian_identities(P, n, m):
    """div grad u = f and vort(n x grad u) = f for the generator's pairs
    (Delta u = f), all on the GPU."""
    print("identities", n, m, flush=True)
    f, u = S.sphere_field(53, 0, n, m, min(n, m) // 8, with_solution=True)
    plan = P.SpherePoisson(n, m, "fp64")
    ug = gpu(u)
    g = plan.tangential_gradient(ug)
    r = plan.curl_scalar(ug)
    d = host(plan.divergence(*g))
    v = host(plan.vorticity(*r))
    plan.close()
    assert rel2(d, f) <= tol2(n, m)
    assert rel2(v, f) <= tol2(n, m)


def test_rossby_haurwitz_vorticity(P):
    """Section 4's example at 10^6 samples: u = n x grad psi for
    psi = cos(theta) + sin(theta)^4 cos(theta) cos(4 lambda); its vorticity is
    Delta psi = -2 cos(theta) - 30 sin(theta)^4 cos(theta) cos(4 lambda)."""
    n = m = 1024
    th = O.theta_grid(m)[:, None]
    lam = O.lambda_grid(n)[None, :]
    psi = np.cos(th) + np.sin(th) ** 4 * np.cos(th) * np.cos(4 * lam)
    lap = -2 * np.cos(th) - 30 * np.sin(th) ** 4 * np.cos(th) * np.cos(4 * lam)
    plan = P.SpherePoisson(n, m, "fp64")
    u = plan.curl_scalar(gpu(psi))
    v = host(plan.vorticity(*u))
    plan.close()
    err = rel2(v, lap)
    print("rossby-haurwitz vorticity rel err", err, flush=True)
    assert err <= tol2(n, m)


def test_vector_calculus_errors(P):
    f = gpu(np.zeros((32, 32)))
    a, b = torch.empty_like(f), torch.empty_like(f)
    plan = P.SpherePoisson(32, 32, "fp64")
    with pytest.raises(P.SpError) as e:
        plan.divergence(f, a, b, out=a)
    assert e.value.code == 6
    with pytest.raises(P.SpError) as e:
        plan.curl(f, a, b, outs=(f, torch.empty_like(f), torch.empty_like(f)))
    assert e.value.code == 6
    plan.close()


def _sum2_integrand(m, n):
    x, y, z = grid_xyz(m, n)
    return 1 + x + y ** 2 + x ** 2 * y + x ** 4 + y ** 5 + (x * y * z) ** 2


@pytest.mark.parametrize("n,m", [(32, 24), (64, 48), (10000, 10000)])
def test_integral_paper_example(P, n, m):
    """Section 4's sum2 example: the integral of 1 + x + y^2 + x^2 y + x^4 + y^5
    + (x y z)^2 over the sphere is 216 pi / 35 (the paper prints
    19.388114662154155); tests/golden/sum2_example.json holds the citation."""
    import json, os
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "sum2_example.json")))
    f = _sum2_integrand(m, n)
    plan = P.SpherePoisson(n, m, "fp64")
    v = float(plan.integral(gpu(f)).cpu())
    plan.close()
    exact = 216 * np.pi / 35
    assert abs(v - exact) <= (1e-13 if n * m < 10 ** 6 else 1e-11) * exact
    assert abs(g["paper_printed_value"] - exact) <= 1e-14


@pytest.mark.parametrize("n,m", [(64, 64), (40, 21), (150, 75), (256, 200)])
def test_integral_matches_oracle(P, n, m):
    f = S.sphere_field(71, 0, n, m, min(n // 2 - 2, m - 3, 30)) + 0.75
    plan = P.SpherePoisson(n, m, "mixed")
    v = float(plan.integral(gpu(f)).cpu())
    plan.close()
    ref = O.sum2(f)
    assert abs(v - ref) <= 1e-13 * abs(ref)


def test_integral_errors(P):
    f = gpu(np.zeros((16, 16)))
    plan = P.SpherePoisson(16, 16, "fp64")
    out = plan.integral(f)
    assert float(out.cpu()) == 0.0
    plan.close()
