"""FP64 oracle of pointwise evaluation of a low-rank function (test infrastructure).

Section 4, "Pointwise evaluation": at a point (x, y, z), projected radially to
the unit sphere, lambda = atan2(y, x) and theta = arccos(z / |p|), and
f = sum_j d_j c_j(theta) r_j(lambda), each factor a 1D Fourier expansion
(eq. FourierExpansions) evaluated in O(m + n) operations.

The factors are given by their samples on the grid (C[j, t] = c_j(theta_t) at
theta_t = (t + 1/2) pi / m, R[j, i] = r_j(lambda_i) at lambda_i = -pi + 2 pi i
/ n).  Their expansions are the trigonometric interpolants of those samples
with the even/odd structure of eq. lowrankRepresentationSplit:

    f = sum_j d_j (c_j^e(theta) r_j^+(lambda) + c_j^o(theta) r_j^-(lambda)),

  c_j^e(theta) = sum_{q=0}^{m-1} alpha_jq cos(q theta)   (cosine interpolant),
  c_j^o(theta) = sum_{q=1}^{m} beta_jq sin(q theta)      (sine interpolant),
  r_j^+- = the even / odd wavenumbers of the real Fourier interpolant of r_j,
           r_j(lambda) = sum_{k=0}^{n/2} w_k Re(h_jk e^{i k (lambda + pi)}),
           h_jk = (1/n) sum_i r_j(lambda_i) e^{-2 pi i k i / n}, w = (1, 2, ..., 2, 1).

At the grid nodes both theta interpolants equal c_j and r_j^+ + r_j^- = r_j,
so the evaluation reproduces the samples.  Here every sum is written out
(explicit cos / sin / exp matrices); the GPU evaluates the same series by
Horner's rule in e^{i theta} and e^{i (lambda + pi)}.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import or call it.
It shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np

from .sphere_poisson import theta_grid

__all__ = ["cosine_coefficients", "sine_coefficients", "lambda_coefficients_real", "point_angles",
           "evaluate_lowrank"]


def cosine_coefficients(C: np.ndarray) -> np.ndarray:
    """alpha [K, m] with C[:, t] = sum_{q=0}^{m-1} alpha_q cos(q theta_t)
    (inverse of the cosine sums on the half-shifted nodes: the nodes make the
    functions cos(q theta) orthogonal with weights m for q = 0, m/2 otherwise)."""
    m = C.shape[1]
    E = np.cos(np.outer(theta_grid(m), np.arange(m)))
    a = (2.0 / m) * (C @ E)
    a[:, 0] *= 0.5
    return a


def sine_coefficients(C: np.ndarray) -> np.ndarray:
    """beta [K, m] (q = 1..m) with C[:, t] = sum_{q=1}^{m} beta_q sin(q theta_t)
    (weights m/2 for q < m and m for q = m, where sin(m theta_t) = (-1)^t)."""
    m = C.shape[1]
    E = np.sin(np.outer(theta_grid(m), np.arange(1, m + 1)))
    b = (2.0 / m) * (C @ E)
    b[:, -1] *= 0.5
    return b


def lambda_coefficients_real(R: np.ndarray) -> np.ndarray:
    """h [K, n/2 + 1]: h_k = (1/n) sum_i R[:, i] e^{-2 pi i k i / n}."""
    n = R.shape[1]
    i = np.arange(n)
    k = np.arange(n // 2 + 1)
    return R @ np.exp(-2j * np.pi * np.outer(i, k) / n) / n


def point_angles(x, y, z):
    """(theta, lambda) of the radial projection of (x, y, z) to the unit sphere."""
    rho = np.sqrt(x * x + y * y + z * z)
    return np.arccos(np.clip(z / rho, -1.0, 1.0)), np.arctan2(y, x)


def evaluate_lowrank(d, C, R, x, y, z) -> np.ndarray:
    """f at the points (x, y, z) from the factors' interpolants (module docstring)."""
    K, m = C.shape
    n = R.shape[1]
    N = n // 2
    th, lam = point_angles(np.asarray(x, float), np.asarray(y, float), np.asarray(z, float))
    alpha = cosine_coefficients(C)
    beta = sine_coefficients(C)
    h = lambda_coefficients_real(R)
    ce = alpha @ np.cos(np.outer(np.arange(m), th))            # [K, P]
    co = beta @ np.sin(np.outer(np.arange(1, m + 1), th))
    k = np.arange(N + 1)
    w = np.full(N + 1, 2.0)
    w[0] = 1.0
    w[N] = 1.0
    E = w[:, None] * np.exp(1j * np.outer(k, lam + np.pi))     # [N+1, P]
    rp = np.real((h * (k % 2 == 0)) @ E)
    rm = np.real((h * (k % 2 == 1)) @ E)
    return np.sum(np.asarray(d, float)[:, None] * (ce * rp + co * rm), axis=0)
