"""Pins of the low-rank input oracle (Section 3, eq. lowrankRepresentation and
lowrankRepresentationSplit; Section 4, Computation of Fourier coefficients,
X = A D B^T): the split reproduces the DFS doubling of the sampled function,
the rank-K coefficient matrix equals the 2D transform of the sampled grid,
1D coefficients of single modes are the textbook ones, and the solve returns
the closed-form solution for spherical harmonics given as rank-2 factors."""
import numpy as np
import pytest

import oracle as O
import oracle.lowrank as OL
import sh_inputs as S
from conftest import rel2


def _coeff_grid(d, C, R):
    """The 2D route of Section 4: doubled samples of sin^2 f, then coeffs2."""
    m = C.shape[1]
    f = OL.lowrank_grid(d, C, R)
    s2 = np.sin(O.doubled_theta_grid(m))[:, None] ** 2
    return O.coeffs2(s2 * O.dfs_double(f), method="dft")


def _random_factors(K, m, n, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal(K), rng.standard_normal((K, m)), rng.standard_normal((K, n))


def test_lowrank_grid_is_the_sum_of_outer_products():
    d, C, R = _random_factors(3, 5, 6, 1)
    f = OL.lowrank_grid(d, C, R)
    ref = sum(d[j] * np.outer(C[j], R[j]) for j in range(3))
    assert np.max(np.abs(f - ref)) <= 1e-14


@pytest.mark.parametrize("K,m,n", [(1, 4, 4), (3, 9, 10), (4, 12, 16), (7, 40, 64)])
def test_split_reproduces_the_doubling(K, m, n):
    """sum_j d_j (c_j^even r_j^+ + c_j^odd r_j^-) on the doubled grid is the
    glide-reflected doubling of eq. BMCsphere of the sampled function."""
    d, C, R = _random_factors(K, m, n, 2 + K)
    ce, co, rp, rm = OL.split_factors(C, R)
    doubled = (ce.T * d) @ rp + (co.T * d) @ rm
    assert np.max(np.abs(doubled - O.dfs_double(OL.lowrank_grid(d, C, R)))) <= 1e-13


def test_single_mode_coefficients():
    """cos(theta) has a_{+-1} = 1/2; sin(2 theta) has a_2 = 1/(2i), a_-2 = -1/(2i);
    cos(3 lambda) has b_{+-3} = 1/2; every other coefficient is zero."""
    m, n = 10, 16
    th2 = O.doubled_theta_grid(m)
    lam = O.lambda_grid(n)
    a = OL.theta_coefficients(np.vstack([np.cos(th2), np.sin(2 * th2)]))
    qs = np.arange(-m, m)
    want = np.zeros((2, 2 * m), dtype=complex)
    want[0, qs == 1] = want[0, qs == -1] = 0.5
    want[1, qs == 2] = 1 / 2j
    want[1, qs == -2] = -1 / 2j
    assert np.max(np.abs(a - want)) <= 1e-15
    b = OL.lambda_coefficients(np.cos(3 * lam)[None, :])
    ks = np.arange(-n // 2, n // 2)
    wb = np.where(np.abs(ks) == 3, 0.5, 0.0)
    assert np.max(np.abs(b[0] - wb)) <= 1e-15


@pytest.mark.parametrize("K,m,n", [(1, 4, 4), (3, 9, 10), (5, 16, 12), (7, 40, 64)])
def test_rank_k_coefficients_equal_2d_transform(K, m, n):
    """X = A D B^T (per parity) from 1D transforms equals the 2D coefficients
    of the sampled grid (any samples: the identity is linearity of the DFT)."""
    d, C, R = _random_factors(K, m, n, 10 + K)
    got = OL.lowrank_coefficients(d, C, R, method="dft")
    ref = _coeff_grid(d, C, R)
    assert np.max(np.abs(got - ref)) <= 1e-14 * max(1.0, np.max(np.abs(ref))) * K


def test_fft_route_equals_dft_route():
    d, C, R = S.lowrank_factors(1, 0, 600, 300, 6, 40)
    a = OL.lowrank_coefficients(d, C, R, method="fft")
    b = OL.lowrank_coefficients(d, C, R, method="dft")
    assert np.max(np.abs(a - b)) <= 1e-14


def _xyz_plus_z_factors(m, n):
    """f = xyz + z as two rank-1 terms: xyz = (sin^2 cos)(theta) (cos sin)(lambda),
    z = cos(theta) * 1; both are spherical harmonics (degrees 3 and 1)."""
    th = O.theta_grid(m)
    lam = O.lambda_grid(n)
    C = np.vstack([np.sin(th) ** 2 * np.cos(th), np.cos(th)])
    R = np.vstack([np.cos(lam) * np.sin(lam), np.ones(n)])
    return np.array([1.0, 1.0]), C, R


@pytest.mark.parametrize("m,n", [(16, 12), (24, 32), (9, 10)])
def test_closed_form_harmonics(m, n):
    """Delta Y_l = -l(l+1) Y_l: u = -xyz/12 - z/2 for f = xyz + z."""
    d, C, R = _xyz_plus_z_factors(m, n)
    x, y, z = S.cartesian(n, m)
    u = OL.solve_lowrank(d, C, R)
    assert np.max(np.abs(u - (-x * y * z / 12 - z / 2))) <= 1e-13


@pytest.mark.parametrize("L,m,n", [(5, 24, 32), (6, 31, 40), (10, 64, 48), (12, 150, 150)])
def test_smooth_field_closed_form_and_dense_route(L, m, n):
    """A band-limited field given as its 2L + 1 (theta profile, lambda mode)
    factors: the low-rank route returns the closed-form solution
    (Delta Y_l = -l(l+1) Y_l) and agrees with the grid route (solve_reduced,
    pinned on its own)."""
    d, C, R, u_exact = S.sphere_field_factors(4, L, n, m, L, with_solution=True)
    assert np.max(np.abs(OL.lowrank_grid(d, C, R) - S.sphere_field(4, L, n, m, L))) <= 1e-13
    u = OL.solve_lowrank(d, C, R)
    assert rel2(u, u_exact) <= 1e-12
    assert rel2(u, O.solve_reduced(OL.lowrank_grid(d, C, R))) <= 1e-12


def test_prescribed_integral():
    """Adding the integral c shifts u by c / (4 pi) (the k = 0 constraint)."""
    d, C, R = S.sphere_field_factors(5, 0, 32, 24, 6)
    u0 = OL.solve_lowrank(d, C, R, 0.0)
    u1 = OL.solve_lowrank(d, C, R, 1.7)
    assert np.max(np.abs(u1 - u0 - 1.7 / (4 * np.pi))) <= 1e-13


def test_pole_singular_factors_leave_the_resolved_class():
    """Random factors (a lambda-dependent value at the poles) make a right-hand
    side whose solution is not resolved: the literal-truncation route and the
    grid route then solve different discrete problems, so the low-rank GPU
    path is compared with the grid route's contract on such inputs."""
    d, C, R = S.lowrank_factors(3, 4, 32, 24, 4, 5)
    f = OL.lowrank_grid(d, C, R)
    d = np.append(d, -O.sum2(f) / (4 * np.pi))
    C = np.vstack([C, np.ones(24)])
    R = np.vstack([R, np.ones(32)])
    u = OL.solve_lowrank(d, C, R)
    assert rel2(u, O.solve_reduced(OL.lowrank_grid(d, C, R))) > 1e-6


def _planted(monkeypatch, split):
    monkeypatch.setattr(OL, "split_factors", split)
    d, C, R = _random_factors(3, 12, 16, 5)
    return float(np.max(np.abs(OL.lowrank_coefficients(d, C, R, method="dft") - _coeff_grid(d, C, R))))


def test_planted_odd_extension_sign(monkeypatch):
    orig = OL.split_factors

    def wrong(C, R):
        ce, co, rp, rm = orig(C, R)
        return ce, np.concatenate([C[:, ::-1], -C], axis=1), rp, rm
    assert _planted(monkeypatch, wrong) > 1e-3


def test_planted_swapped_lambda_parts(monkeypatch):
    orig = OL.split_factors

    def wrong(C, R):
        ce, co, rp, rm = orig(C, R)
        return ce, co, rm, rp
    assert _planted(monkeypatch, wrong) > 1e-3


def test_planted_unreflected_theta(monkeypatch):
    orig = OL.split_factors

    def wrong(C, R):
        ce, co, rp, rm = orig(C, R)
        return np.concatenate([C, C], axis=1), co, rp, rm
    assert _planted(monkeypatch, wrong) > 1e-3
