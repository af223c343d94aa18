"""Pins of the tangential-derivative oracle (Section 4, eq. diff_x/y/z, dfdx,
Msin) against closed forms that do not come from the oracle: the surface
gradient of the restriction of a polynomial F(x, y, z) is
grad F - (p . grad F) p, and the paper's worked example
d^t cos(theta)/dx = -x z."""
import numpy as np
import pytest

import oracle as O
import oracle.calculus as OC
import sh_inputs as S
from conftest import rel2


def _grid_xyz(m, n):
    th = O.theta_grid(m)[:, None]
    lam = O.lambda_grid(n)[None, :]
    return np.cos(lam) * np.sin(th), np.sin(lam) * np.sin(th), np.cos(th) * np.ones_like(lam)


def _rel3(a, b):
    num = sum(np.linalg.norm(x - y) ** 2 for x, y in zip(a, b))
    den = sum(np.linalg.norm(y) ** 2 for y in b)
    return float(np.sqrt(num / den))


# a random quartic: F = sum c_abc x^a y^b z^c over a + b + c <= 4
_EXPS = [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c <= 4]
_COEF = np.random.default_rng(7).standard_normal(len(_EXPS))


def _quartic(x, y, z):
    return sum(c * x ** a * y ** b * z ** e for c, (a, b, e) in zip(_COEF, _EXPS))


def _quartic_grad(x, y, z):
    gx = sum(c * a * x ** max(a - 1, 0) * y ** b * z ** e for c, (a, b, e) in zip(_COEF, _EXPS) if a)
    gy = sum(c * b * x ** a * y ** max(b - 1, 0) * z ** e for c, (a, b, e) in zip(_COEF, _EXPS) if b)
    gz = sum(c * e * x ** a * y ** b * z ** max(e - 1, 0) for c, (a, b, e) in zip(_COEF, _EXPS) if e)
    return gx, gy, gz


def test_paper_example_cos_theta():
    """Section 4: applying d^t/dx to cos(theta) gives -x z on the sphere; the
    other components of the surface gradient of z are -y z and 1 - z^2."""
    m, n = 12, 16
    x, y, z = _grid_xyz(m, n)
    gx, gy, gz = O.tangential_gradient(z.copy())
    assert np.max(np.abs(gx + x * z)) <= 1e-13
    assert np.max(np.abs(gy + y * z)) <= 1e-13
    assert np.max(np.abs(gz - (1 - z * z))) <= 1e-13


@pytest.mark.parametrize("m,n", [(12, 16), (9, 10), (16, 12), (31, 40)])
def test_quartic_closed_form(m, n):
    x, y, z = _grid_xyz(m, n)
    got = O.tangential_gradient(_quartic(x, y, z))
    ref = O.polynomial_surface_gradient(_quartic_grad, m, n)
    assert _rel3(got, ref) <= 1e-12


def test_gradient_is_tangent():
    m, n = 40, 48
    f = S.sphere_field(31, 0, n, m, 12)
    gx, gy, gz = O.tangential_gradient(f)
    x, y, z = _grid_xyz(m, n)
    scale = np.sqrt(np.mean(gx ** 2 + gy ** 2 + gz ** 2))
    assert np.max(np.abs(x * gx + y * gy + z * gz)) <= 1e-12 * scale


def test_dirichlet_energy_identity():
    """Green's identity on the closed sphere: for u with Delta u = f, the
    integral of |grad_s u|^2 equals minus the integral of u f.  u and f are
    the generator's closed-form pair (f a band-limited harmonic field,
    u = -sum c Y / (l (l + 1))); the integrals use the paper's quadrature
    (sum2), exact for these band limits."""
    m, n, L = 48, 64, 10
    f, u = S.sphere_field(33, 0, n, m, L, with_solution=True)
    gx, gy, gz = O.tangential_gradient(u)
    lhs = O.surface_integral(gx * gx + gy * gy + gz * gz)
    rhs = -O.surface_integral(u * f)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_planted_transposed_msin_is_caught(monkeypatch):
    real = OC.msin_matrix
    monkeypatch.setattr(OC, "msin_matrix", lambda M: real(M).T)
    m, n = 12, 16
    x, y, z = _grid_xyz(m, n)
    got = OC.tangential_gradient(_quartic(x, y, z))
    ref = OC.polynomial_surface_gradient(_quartic_grad, m, n)
    assert _rel3(got, ref) > 1e-3


def test_planted_reversed_sine_shift_is_caught(monkeypatch):
    real = OC._times_sin
    monkeypatch.setattr(OC, "_times_sin", lambda C, axis: -real(C, axis))
    m, n = 12, 16
    x, y, z = _grid_xyz(m, n)
    got = OC.tangential_gradient(_quartic(x, y, z))
    ref = OC.polynomial_surface_gradient(_quartic_grad, m, n)
    assert _rel3(got, ref) > 1e-3


def test_planted_printed_z_sign_is_caught():
    """The z component with the sign as printed (+sin(theta) d/dtheta) fails
    the closed form: the minus sign is the chain rule's."""
    m, n = 12, 16
    x, y, z = _grid_xyz(m, n)
    gx, gy, gz = O.tangential_gradient(_quartic(x, y, z))
    ref = O.polynomial_surface_gradient(_quartic_grad, m, n)
    assert _rel3((gx, gy, -gz), ref) > 1e-3


def test_refined_grid_agrees_on_common_rows():
    """The same band-limited field sampled with 3m rows contains the m-row
    nodes (theta at rows 3j + 1): the gradient there must agree (a property of
    the exact result, independent of the grid)."""
    n, m, L = 150, 75, 40
    a = O.tangential_gradient(S.sphere_field(41, 0, n, m, L))
    b = O.tangential_gradient(S.sphere_field(41, 0, n, 3 * m, L))
    assert _rel3(a, tuple(c[1::3] for c in b)) <= 1e-13


def _tol2(n, m):
    """Two spectral differentiations: the rounding floor eps |f| of the
    transforms is amplified twice by the gain of one (max(n/2, m) sqrt(m))."""
    k = max(n // 2, m) * np.sqrt(m)
    return max(1e-11, np.finfo(np.float64).eps * k * k)


@pytest.mark.parametrize("n,m,L", [(48, 40, 10), (64, 33, 12)])
def test_vector_identities_on_poisson_pairs(n, m, L):
    """For the generator's pairs (Delta u = f): div grad u = f and
    vort(n x grad u) = f (both are the surface Laplacian); vort grad u = 0 and
    div(n x grad u) = 0."""
    f, u = S.sphere_field(51, 0, n, m, L, with_solution=True)
    g = O.tangential_gradient(u)
    r = O.curl_scalar(u)
    tol = _tol2(n, m)
    scale = np.max(np.abs(f))
    assert rel2(O.divergence(*g), f) <= tol
    assert rel2(O.vorticity(*r), f) <= tol
    assert np.max(np.abs(O.vorticity(*g))) <= tol * scale
    assert np.max(np.abs(O.divergence(*r))) <= tol * scale


def test_rossby_haurwitz_vorticity():
    """Section 4's example: u = n x grad psi for the Rossby-Haurwitz stream
    function psi = cos(theta) + sin(theta)^4 cos(theta) cos(4 lambda), a sum of
    a degree-1 and a degree-5 harmonic, so vort u = Delta psi
    = -2 cos(theta) - 30 sin(theta)^4 cos(theta) cos(4 lambda)."""
    n, m = 64, 48
    th = O.theta_grid(m)[:, None]
    lam = O.lambda_grid(n)[None, :]
    psi = np.cos(th) + np.sin(th) ** 4 * np.cos(th) * np.cos(4 * lam)
    lap = -2 * np.cos(th) - 30 * np.sin(th) ** 4 * np.cos(th) * np.cos(4 * lam)
    assert rel2(O.vorticity(*O.curl_scalar(psi)), lap) <= _tol2(n, m)


def test_curl_components_against_definition():
    """The surface curl of a gradient field is tangent (n . curl is the
    vorticity, zero here) and its components follow the paper's formula."""
    n, m = 32, 24
    f = S.sphere_field(52, 0, n, m, 8)
    gx, gy, gz = O.tangential_gradient(f)
    cx, cy, cz = O.curl(gx, gy, gz)
    x, y, z = _grid_xyz(m, n)
    assert np.max(np.abs(x * cx + y * cy + z * cz)) <= _tol2(n, m) * np.max(np.abs(f))
