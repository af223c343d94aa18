"""Pins of the CPU oracle against facts that do not come from the oracle itself:
values the paper prints, closed-form solutions, textbook identities, library
routines for sub-steps, brute force on tiny inputs.  The last group plants
plausible mistakes in the oracle (monkeypatched, CPU only) and checks that a
pin catches each of them."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla

import oracle as O
import sh_inputs as S
from conftest import rel2

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


# ---------------------------------------------------------------- paper values

def test_sum2_worked_example():
    """Section 4 (Integration): the integral of 1+x+y^2+x^2y+x^4+y^5+(xyz)^2 over
    the sphere is 216 pi/35; the paper prints 19.388114662154155 with error
    3.553e-15.  The oracle's coefficient-space integral must reproduce it."""
    g = _golden("sum2_example.json")
    exact = 216.0 * np.pi / 35.0
    assert abs(g["paper_printed_value"] - exact) <= 4e-15
    for n, m in [(32, 16), (20, 10), (64, 33), (14, 9)]:
        x, y, z = S.cartesian(n, m)
        f = 1 + x + y ** 2 + x ** 2 * y + x ** 4 + y ** 5 + (x * y * z) ** 2
        val = O.sum2(f)
        assert abs(val - exact) <= 1e-13, (n, m, val)


def test_msin_eigenvalues():
    """Footnote to eq. (Msin): eig(M_sin) = cos(pi l/(m+1)), l = 1..m."""
    g = _golden("msin_eigenvalues.json")
    for mp in g["orders"]:
        _, _, Msin = O.coefficient_operators(mp)
        ev = np.sort(np.linalg.eigvalsh(Msin))
        ref = np.sort(np.cos(np.pi * np.arange(1, mp + 1) / (mp + 1)))
        assert np.max(np.abs(ev - ref)) <= 1e-14
        assert np.min(np.abs(ev)) > 0  # invertible for even order


# ---------------------------------------------------------------- sub-steps

def test_dfs_doubling_is_the_sphere_function():
    """The doubled function on theta in (-pi, 0) is the same point of the sphere:
    (lambda, -theta) and (lambda + pi, theta) have equal (x, y, z)."""
    n, m = 12, 7
    lam = O.lambda_grid(n)
    th2 = O.doubled_theta_grid(m)
    L, T = np.meshgrid(lam, th2)

    def g(x, y, z):
        return np.exp(x) * np.cos(3 * y) + z ** 3 * x

    direct = g(np.cos(L) * np.sin(T), np.sin(L) * np.sin(T), np.cos(T))
    x, y, z = S.cartesian(n, m)
    assert np.max(np.abs(O.dfs_double(g(x, y, z)) - direct)) <= 1e-14


def test_coeffs2_direct_sum_vs_fft():
    rng = np.random.default_rng(5)
    for m2, n in [(8, 6), (16, 10), (30, 8)]:
        gt = rng.standard_normal((m2, n))
        a = O.coeffs2(gt, "dft")
        b = O.coeffs2(gt, "fft")
        assert np.max(np.abs(a - b)) <= 1e-14
        # and sampling inverts it on the original rows
        back = O.sample2(a, O.doubled_theta_grid(m2 // 2)[m2 // 2:], n, "dft")
        assert np.max(np.abs(back - gt[m2 // 2:])) <= 1e-13


def test_bmc_coefficient_parity():
    """Column k of the doubled function has parity (-1)^k in theta
    (Section 3.2 even/odd split): X_{-q,k} = (-1)^k X_{q,k}."""
    n, m = 16, 12
    f = S.sphere_field(99, 0, n, m, 5)
    X = O.coeffs2(O.dfs_double(f))
    qs = np.arange(-m, m)
    ks = np.arange(-n // 2, n // 2)
    for iq, q in enumerate(qs):
        if q == -m:
            continue
        jq = np.where(qs == -q)[0][0]
        assert np.max(np.abs(X[jq] - ((-1.0) ** ks) * X[iq])) <= 1e-14


def test_operator_bands_from_the_differential_operator():
    """Apply sin^2 d^2/dtheta^2 + cos sin d/dtheta to e^{iq theta} on a fine grid
    and project back: the coefficients sit at q-2, q, q+2 and equal the bands
    used by both oracle modes."""
    th = 2 * np.pi * np.arange(64) / 64
    for q in [-5, -2, -1, 0, 1, 3, 7]:
        e = np.exp(1j * q * th)
        Le = np.sin(th) ** 2 * (-q * q) * e + np.cos(th) * np.sin(th) * (1j * q) * e
        c = np.fft.fft(Le) / 64
        for p in range(-20, 21):
            val = c[p % 64]
            sub, diag, sup = O.reduced_bands(np.array([p]), 0.0)
            if p == q:
                want = diag[0]
            elif p == q + 2:
                want = sub[0]       # row p, column p-2
            elif p == q - 2:
                want = sup[0]       # row p, column p+2
            else:
                want = 0.0
            assert abs(val - want) <= 1e-13, (q, p, val, want)


def test_sylvester_product_matches_bands_in_the_interior():
    """The paper's L = M_sin^2 D^2 + M_cos M_sin D has only offsets 0, +-2 and its
    interior rows equal the band formulas; two edge diagonals differ."""
    mp = 24
    L = O.sylvester_operator(mp)
    q = np.arange(-mp // 2, mp // 2)
    offs = {d for d in range(-mp + 1, mp) if np.max(np.abs(np.diag(L, d))) > 0}
    assert offs <= {-2, 0, 2}
    sub, diag, sup = O.reduced_bands(q, 0.0)
    inner = slice(2, mp - 2)
    assert np.max(np.abs(np.diag(L)[inner] - diag[inner])) <= 1e-12
    assert np.max(np.abs(np.diag(L, -2)[1:-1] - sub[2:][1:-1])) <= 1e-12
    assert np.max(np.abs(np.diag(L, 2)[1:-1] - sup[:-2][1:-1])) <= 1e-12


def test_own_thomas_vs_library_banded_solver():
    rng = np.random.default_rng(3)
    n = 40
    sub = rng.uniform(0.1, 1.0, n)
    sup = rng.uniform(0.1, 1.0, n)
    diag = -(sub + sup + rng.uniform(0.0, 0.5, n))
    rhs = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    ab = np.zeros((3, n))
    ab[0, 1:] = sup[:-1]
    ab[1] = diag
    ab[2, :-1] = sub[1:]
    ref = sla.solve_banded((1, 1), ab, rhs)
    got = O.thomas(sub[:, None], diag[:, None], sup[:, None], rhs)
    assert np.max(np.abs(got - ref)) <= 1e-13


def test_cos_sin_transforms_vs_explicit_sums():
    rng = np.random.default_rng(4)
    for m in [5, 8, 13]:
        th = O.theta_grid(m)
        x = rng.standard_normal((m, 2))
        Phi = np.cos(np.outer(th, np.arange(m)))
        Psi = np.sin(np.outer(th, np.arange(1, m + 1)))
        a = O.cos_analysis(x)
        b = O.sin_analysis(x)
        assert np.max(np.abs(Phi @ a - x)) <= 1e-13
        assert np.max(np.abs(Psi @ b - x)) <= 1e-13
        assert np.max(np.abs(O.cos_synthesis(a) - Phi @ a)) <= 1e-13
        assert np.max(np.abs(O.sin_synthesis(b) - Psi @ b)) <= 1e-13


# ---------------------------------------------------------------- whole solver

@pytest.mark.parametrize("mode", ["reduced", "literal"])
def test_textbook_solutions(mode):
    """x, z (l = 1, Delta = -2) and xy (l = 2, Delta = -6) have closed-form
    inverses; these catch a wrong sign of k^2 or of the first-order term."""
    solve = O.solve_reduced if mode == "reduced" else O.solve_literal
    n, m = 16, 12
    x, y, z = S.cartesian(n, m)
    for u, lam in [(x, -2.0), (z, -2.0), (x * y, -6.0), (y * z, -6.0), (x * x - y * y, -6.0)]:
        got = solve(lam * u, 0.0)
        assert rel2(got, u) <= 1e-13


@pytest.mark.parametrize("mode", ["reduced", "literal"])
@pytest.mark.parametrize("n,m,L", [(64, 64, 16), (40, 21, 8), (30, 48, 12)])
def test_closed_form_band_limited(mode, n, m, L):
    """Delta^{-1} Y_l^M = -Y_l^M / (l(l+1)) for random band-limited fields
    (l + 2 < m, l < n/2): the discrete solution is exact up to rounding."""
    solve = O.solve_reduced if mode == "reduced" else O.solve_literal
    f, u = S.sphere_field(0, 0, n, m, L, with_solution=True)
    assert rel2(solve(f, 0.0), u) <= 1e-12


def test_closed_form_1m_dof_reduced():
    f, u = S.sphere_field(1, 0, 1024, 1024, 256, with_solution=True)
    assert rel2(O.solve_reduced(f, 0.0), u) <= 1e-12


@pytest.mark.slow
def test_closed_form_1m_dof_literal():
    f, u = S.sphere_field(1, 0, 1024, 1024, 256, with_solution=True)
    assert rel2(O.solve_literal(f, 0.0), u) <= 1e-12


@pytest.mark.parametrize("mode", ["reduced", "literal"])
def test_integral_constraint(mode):
    """The k = 0 row fixes the integral of u: with value c the solution shifts by
    the constant c / (4 pi) (Section 5, eq. integralConstraint2)."""
    solve = O.solve_reduced if mode == "reduced" else O.solve_literal
    n, m, L = 32, 24, 8
    f, u = S.sphere_field(2, 0, n, m, L, with_solution=True)
    for c in [0.0, 1.0, -3.25]:
        got = solve(f, c)
        assert np.max(np.abs(got - (u + c / (4 * np.pi)))) <= 1e-13
        assert abs(O.sum2(got) - c) <= 1e-12


def test_solution_constant_at_the_poles():
    """The solution is BMC-I (Section 5): its limit at each pole is one value.
    Evaluating the reduced solution's coefficients at theta = 0 and pi gives a
    lambda-independent value."""
    n, m, L = 32, 24, 10
    f = S.sphere_field(3, 0, n, m, L)
    u = O.solve_reduced(f)
    # trigonometric interpolation of each lambda-column to theta = 0 via the
    # literal coefficients of the doubled solution
    X = O.coeffs2(O.dfs_double(u))
    pole = np.real(O.sample2(X, np.array([0.0, np.pi]), n, "dft"))
    assert np.ptp(pole[0]) <= 1e-12 * np.max(np.abs(u))
    assert np.ptp(pole[1]) <= 1e-12 * np.max(np.abs(u))


def test_literal_and_reduced_agree_on_resolved_fields():
    rng = np.random.default_rng(7)
    for n, m in [(48, 32), (64, 64), (150, 75)]:
        L = min(n // 2, m) - 4
        f = S.synth(n, m, L, [S.draw_coeffs(L, [7, n, m])])[0]
        assert rel2(O.solve_literal(f), O.solve_reduced(f)) <= 1e-12
    # the paper's sin(50xyz) example (m_p = n = 150), zero mean because it is odd
    x, y, z = S.cartesian(150, 75)
    f = np.sin(50 * x * y * z)
    assert abs(O.sum2(f)) <= 1e-12
    ul, ur = O.solve_literal(f), O.solve_reduced(f)
    assert rel2(ul, ur) <= 1e-6   # agree up to the field's own truncation level


def test_dense_and_banded_literal_agree():
    n, m = 16, 20
    f = S.sphere_field(4, 0, n, m, 6)
    assert rel2(O.solve_literal(f, 0.5, solver="dense"), O.solve_literal(f, 0.5, solver="banded")) <= 1e-13


def test_reduced_tridiagonals_vs_dense_lu():
    """Each per-k tridiagonal solve equals a dense LU solve of the assembled
    (L - k^2) matrix in the same cosine / sine basis."""
    m = 14
    rng = np.random.default_rng(8)
    for sine, ks in [(False, np.array([2, 4, 6])), (True, np.array([1, 3, 9]))]:
        C = rng.standard_normal((m, ks.size))
        got = O.sphere_poisson._solve_columns(C, ks, sine=sine, integral=0.0)
        qs = np.arange(1, m + 1) if sine else np.arange(m)
        for c, k in enumerate(ks):
            A = np.zeros((m, m))
            for r, p in enumerate(qs):
                sub, diag, sup = O.reduced_bands(np.array([p]), k)
                A[r, r] = diag[0]
                if r - 2 >= 0:
                    A[r, r - 2] = sub[0]
                if r + 2 < m:
                    A[r, r + 2] = sup[0]
            ref = np.linalg.solve(A, C[:, c])
            assert np.max(np.abs(got[:, c] - ref)) <= 1e-13 * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("n,m", [(8, 8), (16, 16), (10, 7), (6, 9)])
def test_adjoint_is_the_dense_transpose(n, m):
    Sd = O.dense_operator(n, m)
    g = np.random.default_rng(n * 100 + m).standard_normal((m, n))
    assert np.max(np.abs(O.adjoint_reduced(g).ravel() - Sd.T @ g.ravel())) <= 1e-13


def test_adjoint_dot_product_medium():
    n, m = 128, 96
    rng = np.random.default_rng(11)
    f = rng.standard_normal((m, n))
    g = rng.standard_normal((m, n))
    lhs = np.vdot(O.solve_reduced(f), g)
    rhs = np.vdot(f, O.adjoint_reduced(g))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_gradient_by_central_differences():
    """loss(f) = ||S f - u_obs||^2 is quadratic, so the central difference along
    v equals <grad, v> up to rounding for any step; grad = 2 S^T (S f - u_obs)."""
    n, m = 64, 48
    f = S.sphere_field(4, 0, n, m, 12)
    u_obs = S.sphere_field(4, 0, n, m, 12, tag=S.TAG_OBS) + S.noise(4, 0, (m, n), 1e-3)
    v = S.direction(4, 0, (m, n))

    def loss(ff):
        r = O.solve_reduced(ff) - u_obs
        return float(np.vdot(r, r))

    grad = 2.0 * O.adjoint_reduced(O.solve_reduced(f) - u_obs)
    h = 0.1 * np.linalg.norm(f) / np.linalg.norm(v)
    fd = (loss(f + h * v) - loss(f - h * v)) / (2 * h)
    assert abs(fd - np.vdot(grad, v)) <= 1e-9 * abs(fd)


# ---------------------------------------------------------------- planted mistakes

def _closed_form_error(solve):
    n, m, L = 32, 24, 8
    f, u = S.sphere_field(5, 0, n, m, L, with_solution=True)
    return rel2(solve(f, 0.0), u)


def test_planted_sign_of_k2_is_caught(monkeypatch):
    good = O.reduced_bands
    monkeypatch.setattr(O.sphere_poisson, "reduced_bands",
                        lambda p, k: (lambda s, d, u: (s, d + 2 * np.asarray(k, float) ** 2, u))(*good(p, k)))
    assert _closed_form_error(O.solve_reduced) > 1e-3


def test_planted_dropped_first_order_term_is_caught(monkeypatch):
    def bands(p, k):
        p = np.asarray(p, dtype=np.float64)
        return (p - 2) ** 2 / 4.0, -p * p / 2.0 - np.asarray(k, float) ** 2, (p + 2) ** 2 / 4.0
    monkeypatch.setattr(O.sphere_poisson, "reduced_bands", bands)
    assert _closed_form_error(O.solve_reduced) > 1e-3


def test_planted_transposed_tridiagonal_is_caught(monkeypatch):
    good = O.thomas

    def transposed(sub, diag, sup, rhs):
        tsub, tsup = O.sphere_poisson._transpose_bands(sub, sup)
        return good(tsub, diag, tsup, rhs)
    monkeypatch.setattr(O.sphere_poisson, "thomas", transposed)
    assert _closed_form_error(O.solve_reduced) > 1e-3


def test_planted_doubling_without_shift_is_caught(monkeypatch):
    def bad(f):
        m, n = f.shape
        out = np.empty((2 * m, n))
        out[m:] = f
        out[:m] = f[::-1]          # reflection without the lambda + pi shift
        return out
    monkeypatch.setattr(O.sphere_poisson, "dfs_double", bad)
    assert _closed_form_error(O.solve_literal) > 1e-8


def test_planted_wrong_weights_are_caught(monkeypatch):
    good = O.integration_weights
    monkeypatch.setattr(O.sphere_poisson, "integration_weights", lambda mp: good(mp) * 1.01)
    x, y, z = S.cartesian(32, 16)
    f = 1 + x + y ** 2 + x ** 2 * y + x ** 4 + y ** 5 + (x * y * z) ** 2
    assert abs(O.sum2(f) - 216 * np.pi / 35) > 1e-3


def test_planted_wrong_constraint_is_caught(monkeypatch):
    """A constraint row that forgets the factor 2 of w_q = 2/(1-q^2) moves the mean."""
    good = O.sphere_poisson._solve_columns

    def bad(C, ks, sine, integral, transpose=False):
        out = good(C, ks, sine, integral, transpose)
        if not sine and ks.size and ks[0] == 0 and not transpose:
            q = np.arange(2, C.shape[0], 2)
            out[0, 0] = integral / (4 * np.pi) - 2.0 * np.dot(1.0 / (1.0 - q ** 2.0), out[q, 0])
        return out
    monkeypatch.setattr(O.sphere_poisson, "_solve_columns", bad)
    assert _closed_form_error(O.solve_reduced) > 1e-8


def test_closed_form_degree_2000():
    """l <= 2000 reaches orders M whose sectoral values (sin theta)^M underflow
    double precision near the poles; the generator must still produce exact
    band-limited fields (regression: dropping them broke the closed form)."""
    f, u = S.sphere_field(2, 0, 4096, 2100, 2000, with_solution=True)
    assert rel2(O.solve_reduced(f, 0.0), u) <= 1e-13
