"""Pins of the pointwise-evaluation oracle (Section 4, Pointwise evaluation;
eq. FourierExpansions, lowrankRepresentationSplit): the interpolants
reproduce the samples at the grid nodes, polynomials given in low-rank form
evaluate to their values anywhere on the sphere, and a band-limited field
given by its factors on one grid evaluates to its samples on another grid."""
import numpy as np
import pytest

import oracle as O
import oracle.evaluate as OE
import oracle.lowrank as OL
import sh_inputs as S


def _random_points(P, seed, radius=1.0):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((3, P))
    v *= radius / np.linalg.norm(v, axis=0)
    return v


@pytest.mark.parametrize("K,m,n", [(1, 4, 4), (3, 9, 10), (5, 16, 12), (7, 40, 64)])
def test_reproduces_the_samples_at_the_nodes(K, m, n):
    rng = np.random.default_rng(K + m)
    d, C, R = rng.standard_normal(K), rng.standard_normal((K, m)), rng.standard_normal((K, n))
    x, y, z = S.cartesian(n, m)
    f = OE.evaluate_lowrank(d, C, R, x.ravel(), y.ravel(), z.ravel()).reshape(m, n)
    assert np.max(np.abs(f - OL.lowrank_grid(d, C, R))) <= 1e-12


def test_single_series_coefficients():
    """cos(3 theta) -> alpha_3 = 1; sin(2 theta) -> beta_2 = 1;
    cos(2 lambda) = cos(2 (lambda + pi)) -> h_2 = 1/2 (weight w_2 = 2)."""
    m, n = 12, 16
    th = O.theta_grid(m)
    a = OE.cosine_coefficients(np.cos(3 * th)[None, :])[0]
    assert abs(a[3] - 1) <= 1e-14 and np.max(np.abs(np.delete(a, 3))) <= 1e-14
    b = OE.sine_coefficients(np.sin(2 * th)[None, :])[0]
    assert abs(b[1] - 1) <= 1e-14 and np.max(np.abs(np.delete(b, 1))) <= 1e-14
    lam = O.lambda_grid(n)
    h = OE.lambda_coefficients_real(np.cos(2 * lam)[None, :])[0]
    assert abs(h[2] - 0.5) <= 1e-14 and np.max(np.abs(np.delete(h, 2))) <= 1e-14


def _poly_factors(m, n):
    """f = x y z + z + x^2 - y  as rank-4 factors of band-limited series:
    xyz = (sin^2 cos)(theta) (sin 2 lambda / 2), z = cos(theta) * 1,
    x^2 = sin^2(theta) cos^2(lambda), -y = -sin(theta) sin(lambda)."""
    th = O.theta_grid(m)
    lam = O.lambda_grid(n)
    C = np.vstack([np.sin(th) ** 2 * np.cos(th), np.cos(th), np.sin(th) ** 2, np.sin(th)])
    R = np.vstack([0.5 * np.sin(2 * lam), np.ones(n), np.cos(lam) ** 2, np.sin(lam)])
    return np.array([1.0, 1.0, 1.0, -1.0]), C, R


def _poly(x, y, z):
    rho = np.sqrt(x * x + y * y + z * z)
    x, y, z = x / rho, y / rho, z / rho
    return x * y * z + z + x * x - y


@pytest.mark.parametrize("m,n", [(8, 8), (12, 16), (31, 40)])
@pytest.mark.parametrize("radius", [1.0, 2.5])
def test_polynomial_anywhere(m, n, radius):
    d, C, R = _poly_factors(m, n)
    x, y, z = _random_points(200, m + n, radius)
    assert np.max(np.abs(OE.evaluate_lowrank(d, C, R, x, y, z) - _poly(x, y, z))) <= 1e-13


def test_poles_and_seam():
    """Points on the axis (lambda is arbitrary there) and on the lambda = +-pi seam."""
    d, C, R = _poly_factors(12, 16)
    x = np.array([0.0, 0.0, -1.0, -1.0, 1e-300])
    y = np.array([0.0, 0.0, 0.0, -0.0, 0.0])
    z = np.array([1.0, -1.0, 0.0, 0.3, -2.0])
    assert np.max(np.abs(OE.evaluate_lowrank(d, C, R, x, y, z) - _poly(x, y, z))) <= 1e-13


@pytest.mark.parametrize("L,m,n,m2,n2", [(5, 12, 16, 17, 24), (10, 24, 32, 9, 40), (12, 31, 30, 50, 64)])
def test_band_limited_field_on_another_grid(L, m, n, m2, n2):
    """sphere_field_factors on one grid, evaluated at the nodes of another
    grid, equals the same seeded field sampled there (exact for L < m, n/2)."""
    d, C, R = S.sphere_field_factors(6, L, n, m, L)
    x, y, z = S.cartesian(n2, m2)
    f = OE.evaluate_lowrank(d, C, R, x.ravel(), y.ravel(), z.ravel()).reshape(m2, n2)
    assert np.max(np.abs(f - S.sphere_field(6, L, n2, m2, L))) <= 1e-12


def _planted_error(monkeypatch, name, fn):
    monkeypatch.setattr(OE, name, fn)
    d, C, R = _poly_factors(12, 16)
    x, y, z = _random_points(50, 3)
    return float(np.max(np.abs(OE.evaluate_lowrank(d, C, R, x, y, z) - _poly(x, y, z))))


def test_planted_unshifted_lambda(monkeypatch):
    orig = OE.point_angles
    assert _planted_error(monkeypatch, "point_angles", lambda x, y, z: (orig(x, y, z)[0], orig(x, y, z)[1] + np.pi)) > 1e-3


def test_planted_cosine_weight(monkeypatch):
    orig = OE.cosine_coefficients

    def wrong(C):
        a = orig(C)
        a[:, 0] *= 2.0
        return a
    assert _planted_error(monkeypatch, "cosine_coefficients", wrong) > 1e-3


def test_planted_parity_pairing(monkeypatch):
    """Pairing the sine interpolant with the even wavenumbers breaks the result."""
    monkeypatch.setattr(OE, "sine_coefficients", lambda C: np.hstack([OE.cosine_coefficients(C)[:, 1:], np.zeros((C.shape[0], 1))]))
    d, C, R = _poly_factors(12, 16)
    x, y, z = _random_points(50, 4)
    assert float(np.max(np.abs(OE.evaluate_lowrank(d, C, R, x, y, z) - _poly(x, y, z)))) > 1e-3
