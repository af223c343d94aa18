"""The seeded input generator: real orthonormal spherical harmonics on the grid."""
import numpy as np
import pytest
from scipy.special import sph_harm_y

import sh_inputs as S


@pytest.mark.parametrize("l,M", [(1, 0), (1, 1), (1, -1), (3, 2), (5, -3), (6, 6), (7, -7)])
def test_single_harmonic_matches_scipy(l, M):
    n, m, L = 16, 12, 7
    lam, th = S.grid(n, m)
    LL, TT = np.meshgrid(lam, th)
    c = np.zeros(S.n_coeffs(L))
    c[l * l - 1 + M + l] = 1.0
    f = S.synth(n, m, L, [c])[0]
    Y = sph_harm_y(l, abs(M), TT, LL)          # complex, Condon-Shortley phase
    if M > 0:
        ref = np.sqrt(2) * (-1) ** M * Y.real
    elif M < 0:
        ref = np.sqrt(2) * (-1) ** M * Y.imag
    else:
        ref = Y.real
    assert np.max(np.abs(f - ref)) <= 1e-14


def test_high_degree_against_scipy_at_sampled_points():
    n, m, L = 64, 41, 30
    rng = np.random.default_rng(0)
    c = S.draw_coeffs(L, [0, 0, 0])
    f = S.synth(n, m, L, [c])[0]
    lam, th = S.grid(n, m)
    for _ in range(5):
        j, i = rng.integers(0, m), rng.integers(0, n)
        val = 0.0
        idx = 0
        for l in range(1, L + 1):
            for M in range(-l, l + 1):
                Y = sph_harm_y(l, abs(M), th[j], lam[i])
                y = np.sqrt(2) * (-1) ** M * (Y.real if M > 0 else Y.imag) if M else Y.real
                val += c[idx] * y
                idx += 1
        assert abs(val - f[j, i]) <= 1e-13


def test_seeding_and_law():
    a = S.draw_coeffs(20, [2, 3, 0])
    b = S.draw_coeffs(20, [2, 3, 0])
    c = S.draw_coeffs(20, [2, 3, 1])
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    assert a.size == 20 * 20 + 2 * 20
    z = a * (1 + S.degrees(20)) ** 2
    assert abs(np.mean(z)) < 0.2 and abs(np.std(z) - 1) < 0.1


def test_orthonormality_by_quadrature():
    # fine grid, Fejer-type check: integral of Y_a Y_b over the sphere
    n, m, L = 64, 64, 4
    lam, th = S.grid(n, m)
    fields = []
    for idx in range(S.n_coeffs(L)):
        c = np.zeros(S.n_coeffs(L))
        c[idx] = 1.0
        fields.append(S.synth(n, m, L, [c])[0])
    F = np.array(fields).reshape(len(fields), -1)
    # exact quadrature for band-limited integrands on the half-shifted grid:
    # weights from the cosine-series integral of sin(theta)
    q = np.arange(0, m, 2)
    wq = 2.0 / (1.0 - q ** 2)
    W = np.array([np.sum(wq * np.cos(q * t) * np.where(q == 0, 1.0, 2.0)) / m for t in th])
    G = (F * np.repeat(W, n)[None, :] * (2 * np.pi / n)) @ F.T
    assert np.max(np.abs(G - np.eye(len(fields)))) <= 1e-13
