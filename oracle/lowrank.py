"""FP64 oracle of the low-rank input path of the Poisson solver (test infrastructure).

A function given in the low-rank form of Section 3 (eq. lowrankRepresentation),

    f(lambda, theta) = sum_{j=1}^{K} d_j c_j(theta) r_j(lambda),

is handed over as samples: C[j, t] = c_j(theta_t) on the m rows of the grid
(theta_t = (t + 1/2) pi / m) and R[j, i] = r_j(lambda_i) on the n columns
(lambda_i = -pi + 2 pi i / n).

The doubled function f~ of the DFS method is again of low rank once the
factors are split as in eq. lowrankRepresentationSplit: with the even and odd
extensions of c_j to (-pi, pi) and the pi-periodic / pi-antiperiodic parts of
r_j (r_j^+- (lambda) = (r_j(lambda) +- r_j(lambda + pi)) / 2),

    f~ = sum_j d_j (c_j^even r_j^+ + c_j^odd r_j^-),

which equals f(lambda + pi, -theta) for theta < 0 (the glide reflection of
eq. BMCsphere).  Section 4 ("Computation of Fourier coefficients") then gives
the 2D coefficient matrix as X = A D B^T from the 1D Fourier coefficients of
the factors (eq. FourierExpansions), K FFTs in each direction instead of a 2D
FFT of the grid; Section 5 notes that this makes forming the right-hand side
O(mn).  Here A holds the theta coefficients of sin(theta)^2 c_j (the solver's
right-hand side is sin(theta)^2 f~), one matrix per parity.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import or call it.
It shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np

from .sphere_poisson import doubled_theta_grid, lambda_grid, sample2, solve_coefficients, theta_grid

__all__ = ["lowrank_grid", "split_factors", "theta_coefficients", "lambda_coefficients",
           "lowrank_coefficients", "solve_lowrank"]


def lowrank_grid(d: np.ndarray, C: np.ndarray, R: np.ndarray) -> np.ndarray:
    """The sampled function f[t, i] = sum_j d_j C[j, t] R[j, i] (eq. lowrankRepresentation)."""
    return (C.T * d[None, :]) @ R


def split_factors(C: np.ndarray, R: np.ndarray):
    """BMC split of the factors (eq. lowrankRepresentationSplit) on the doubled
    theta grid theta'_u = (u - m + 1/2) pi / m, u = 0..2m-1: row u < m sits at
    -theta_{m-1-u}.  Returns (c_even, c_odd) of shape [K, 2m] and
    (r_plus, r_minus) of shape [K, n]."""
    m = C.shape[1]
    n = R.shape[1]
    if n % 2:
        raise ValueError("n must be even (lambda + pi must be a grid point)")
    c_even = np.concatenate([C[:, ::-1], C], axis=1)
    c_odd = np.concatenate([-C[:, ::-1], C], axis=1)
    shifted = np.roll(R, -n // 2, axis=1)          # r(lambda_i + pi) = r(lambda_{i + n/2})
    return c_even, c_odd, 0.5 * (R + shifted), 0.5 * (R - shifted)


def theta_coefficients(c2: np.ndarray, method: str = "auto") -> np.ndarray:
    """a_q = (1/2m) sum_u c(theta'_u) e^{-i q theta'_u}, q = -m..m-1, for each
    row of c2 ([K, 2m]); the theta half of eq. FourierExpansions."""
    m2 = c2.shape[1]
    qs = np.arange(-m2 // 2, m2 // 2)
    if method == "auto":
        method = "dft" if m2 <= 512 else "fft"
    if method == "dft":
        return c2 @ np.exp(-1j * np.outer(doubled_theta_grid(m2 // 2), qs)) / m2
    # theta'_u = -pi + 2 pi (u + 1/2) / (2m)
    G = np.fft.fft(c2, axis=1)[:, np.mod(qs, m2)] / m2
    return G * (np.exp(1j * np.pi * qs) * np.exp(-1j * np.pi * qs / m2))[None, :]


def lambda_coefficients(r: np.ndarray, method: str = "auto") -> np.ndarray:
    """b_k = (1/n) sum_i r(lambda_i) e^{-i k lambda_i}, k = -n/2..n/2-1, for
    each row of r ([K, n]); the lambda half of eq. FourierExpansions."""
    n = r.shape[1]
    ks = np.arange(-n // 2, n // 2)
    if method == "auto":
        method = "dft" if n <= 512 else "fft"
    if method == "dft":
        return r @ np.exp(-1j * np.outer(lambda_grid(n), ks)) / n
    G = np.fft.fft(r, axis=1)[:, np.mod(ks, n)] / n   # lambda_i = -pi + 2 pi i / n
    return G * np.exp(1j * np.pi * ks)[None, :]


def lowrank_coefficients(d: np.ndarray, C: np.ndarray, R: np.ndarray, method: str = "auto") -> np.ndarray:
    """Coefficient matrix F of sin(theta)^2 f~ ([2m, n], the layout of
    ``coeffs2``) as X = A D B^T per parity: A columns are the theta
    coefficients of sin^2 c_j^even and sin^2 c_j^odd, B columns the lambda
    coefficients of r_j^+ and r_j^- (Section 4, Computation of Fourier
    coefficients)."""
    m = C.shape[1]
    c_even, c_odd, r_plus, r_minus = split_factors(C, R)
    s2 = np.sin(doubled_theta_grid(m)) ** 2
    A_even = theta_coefficients(c_even * s2[None, :], method).T     # [2m, K]
    A_odd = theta_coefficients(c_odd * s2[None, :], method).T
    B_plus = lambda_coefficients(r_plus, method).T                  # [n, K]
    B_minus = lambda_coefficients(r_minus, method).T
    D = np.diag(np.asarray(d, dtype=np.float64))
    return A_even @ D @ B_plus.T + A_odd @ D @ B_minus.T


def solve_lowrank(d: np.ndarray, C: np.ndarray, R: np.ndarray, integral: float = 0.0,
                  solver: str = "auto") -> np.ndarray:
    """Poisson on the sphere with a low-rank right-hand side: F from the
    factors (``lowrank_coefficients``), then the Section 5 solve on
    coefficients and the evaluation on the m original rows."""
    m = C.shape[1]
    n = R.shape[1]
    F = lowrank_coefficients(d, C, R)
    X = solve_coefficients(F, integral, solver)
    method = "dft" if max(2 * m, n) <= 256 else "fft"
    return np.real(sample2(X, theta_grid(m), n, method))
