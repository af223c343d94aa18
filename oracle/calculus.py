"""FP64 oracle of the tangential derivatives on the sphere (test infrastructure).

Section 4, "Differentiation": the Cartesian components of the surface
gradient are, by the chain rule,

    d^t/dx = -(sin(lambda)/sin(theta)) d/dlambda + cos(lambda) cos(theta) d/dtheta
    d^t/dy =  (cos(lambda)/sin(theta)) d/dlambda + sin(lambda) cos(theta) d/dtheta
    d^t/dz = -sin(theta) d/dtheta

(eq. diff_x, diff_y, diff_z).  The paper prints the z component with a plus
sign; the chain rule with z = cos(theta) gives the minus sign, which is also
the only sign for which the gradient is tangent to the sphere (x g_x + y g_y
+ z g_z = 0).  This module takes the minus sign.

The computation follows the paper's coefficient-space algorithm (eq. dfdx
and eq. Msin) on the full 2D Fourier coefficient matrix of the doubled
function, not the grid: derivatives multiply coefficients by i k and i q,
multiplication by cos/sin of lambda or theta shifts them by one mode (the
expansions grow by one mode on each side), and the division by sin(theta) is
a solve with the truncated multiplication matrix M_sin, which is invertible
because the doubled theta range has an even number of modes.  The result is
evaluated on the original rows by explicit sums.

Nyquist modes (q = -m of the doubled theta range, k = -n/2) have no partner
in the truncated range; their derivatives are set to zero.  For band-limited
input (no energy there) every step is exact.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import or call it.
It shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np

from .sphere_poisson import coeffs2, dfs_double, lambda_grid, theta_grid

__all__ = ["msin_matrix", "tangential_gradient", "polynomial_surface_gradient", "curl_scalar", "divergence",
           "curl", "vorticity"]


def msin_matrix(M: int) -> np.ndarray:
    """Multiplication by sin(theta) on the coefficients of e^{i q theta},
    q = -M/2..M/2-1, truncated to that range (eq. Msin):
    (M_sin a)_q = (i/2)(a_{q+1} - a_{q-1})."""
    S = np.zeros((M, M), dtype=np.complex128)
    for r in range(M):
        if r + 1 < M:
            S[r, r + 1] = 0.5j
        if r - 1 >= 0:
            S[r, r - 1] = -0.5j
    return S


def _times_cos(C: np.ndarray, axis: int) -> np.ndarray:
    """cos(.) * sum_j C_j e^{i j .}: coefficient j of the product is
    (C_{j-1} + C_{j+1}) / 2; the index range grows by one on each side."""
    C = np.moveaxis(C, axis, 0)
    out = np.zeros((C.shape[0] + 2,) + C.shape[1:], dtype=np.complex128)
    out[2:] += 0.5 * C      # C_{j-1} lands on j (shifted by the new lower end)
    out[:-2] += 0.5 * C     # C_{j+1} lands on j
    return np.moveaxis(out, 0, axis)


def _times_sin(C: np.ndarray, axis: int) -> np.ndarray:
    """sin(.) * sum_j C_j e^{i j .}: coefficient j is (C_{j-1} - C_{j+1}) / (2i)."""
    C = np.moveaxis(C, axis, 0)
    out = np.zeros((C.shape[0] + 2,) + C.shape[1:], dtype=np.complex128)
    out[2:] += C / 2j
    out[:-2] -= C / 2j
    return np.moveaxis(out, 0, axis)


def _pad(C: np.ndarray, axis: int, lo: int, hi: int) -> np.ndarray:
    pad = [(0, 0)] * C.ndim
    pad[axis] = (lo, hi)
    return np.pad(C, pad)


def _evaluate(C: np.ndarray, q0: int, k0: int, thetas: np.ndarray, lams: np.ndarray) -> np.ndarray:
    """Real part of sum_{q,k} C[q - q0, k - k0] e^{i q theta} e^{i k lambda} by explicit sums."""
    qs = q0 + np.arange(C.shape[0])
    ks = k0 + np.arange(C.shape[1])
    return (np.exp(1j * np.outer(thetas, qs)) @ C @ np.exp(1j * np.outer(ks, lams))).real


def tangential_gradient(f: np.ndarray) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """(d^t f/dx, d^t f/dy, d^t f/dz) on the grid of f ([m, n], n even):
    samples f[j, i] at theta_j = (j + 1/2) pi / m, lambda_i = -pi + 2 pi i / n."""
    m, n = f.shape
    M = 2 * m
    # q = -m..m-1 rows, k = -n/2..n/2-1 columns.  The FFT evaluation (the
    # paper's route, Section 4 "Computation of Fourier coefficients"): the
    # explicit sums round the phase q theta to about q theta eps, an error the
    # derivative then multiplies by q (1e-12 at m = 75).
    X = coeffs2(dfs_double(f), method="fft")
    qs = np.arange(-m, m)
    ks = np.arange(-n // 2, n // 2)
    dq = 1j * qs.astype(np.float64)
    dk = 1j * ks.astype(np.float64)
    dq[0] = 0.0                                     # q = -m has no partner
    dk[0] = 0.0                                     # k = -n/2 has no partner
    F_lam = X * dk[None, :]                          # d f / d lambda
    F_th = X * dq[:, None]                           # d f / d theta
    # (d f / d lambda) / sin(theta): solve with M_sin column by column (eq. Msin)
    A = np.linalg.solve(msin_matrix(M), F_lam)
    # bring every term to the common index range q = -m-1..m, k = -n/2-1..n/2
    A_q = _pad(A, 0, 1, 1)
    sinl_A = _times_sin(A_q, 1)
    cosl_A = _times_cos(A_q, 1)
    cost_F = _times_cos(F_th, 0)
    sint_F = _pad(_times_sin(F_th, 0), 1, 1, 1)
    cosl_cost_F = _times_cos(cost_F, 1)
    sinl_cost_F = _times_sin(cost_F, 1)
    Gx = -sinl_A + cosl_cost_F
    Gy = cosl_A + sinl_cost_F
    Gz = -sint_F
    th = theta_grid(m)
    lam = lambda_grid(n)
    q0, k0 = -m - 1, -n // 2 - 1
    return (_evaluate(Gx, q0, k0, th, lam), _evaluate(Gy, q0, k0, th, lam),
            _evaluate(Gz, q0, k0, th, lam))


def polynomial_surface_gradient(grad_F, m: int, n: int):
    """Closed form for a function that is the restriction of a smooth F(x, y, z):
    grad_s f = grad F - (p . grad F) p at the point p = (x, y, z) of the unit
    sphere.  grad_F(x, y, z) returns the three partial derivatives of F."""
    th = theta_grid(m)[:, None]
    lam = lambda_grid(n)[None, :]
    x = np.cos(lam) * np.sin(th)
    y = np.sin(lam) * np.sin(th)
    z = np.cos(th) * np.ones_like(lam)
    Fx, Fy, Fz = (np.broadcast_to(v, x.shape) for v in grad_F(x, y, z))
    radial = x * Fx + y * Fy + z * Fz
    return Fx - radial * x, Fy - radial * y, Fz - radial * z


def _point(m: int, n: int):
    th = theta_grid(m)[:, None]
    lam = lambda_grid(n)[None, :]
    return np.cos(lam) * np.sin(th), np.sin(lam) * np.sin(th), np.cos(th) * np.ones_like(lam)


def curl_scalar(f: np.ndarray):
    """n x grad f with n = p = (x, y, z) (Section 4, eq. CurlScalarF)."""
    gx, gy, gz = tangential_gradient(f)
    x, y, z = _point(*f.shape)
    return y * gz - z * gy, z * gx - x * gz, x * gy - y * gx


def divergence(fx: np.ndarray, fy: np.ndarray, fz: np.ndarray) -> np.ndarray:
    """d^t fx/dx + d^t fy/dy + d^t fz/dz (Section 4, Vector calculus)."""
    return tangential_gradient(fx)[0] + tangential_gradient(fy)[1] + tangential_gradient(fz)[2]


def curl(fx: np.ndarray, fy: np.ndarray, fz: np.ndarray):
    """(d^t fz/dy - d^t fy/dz, d^t fx/dz - d^t fz/dx, d^t fy/dx - d^t fx/dy)."""
    gx, gy, gz = tangential_gradient(fx), tangential_gradient(fy), tangential_gradient(fz)
    return gz[1] - gy[2], gx[2] - gz[0], gy[0] - gx[1]


def vorticity(fx: np.ndarray, fy: np.ndarray, fz: np.ndarray) -> np.ndarray:
    """n . curl f (Section 4, Vector calculus)."""
    cx, cy, cz = curl(fx, fy, fz)
    x, y, z = _point(*fx.shape)
    return x * cx + y * cy + z * cz
