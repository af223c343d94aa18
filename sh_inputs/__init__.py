"""Seeded synthetic inputs shared by the tests, the oracle checks and the bench.

This module makes right-hand sides and nothing else: band-limited random
fields built from real, orthonormal spherical harmonics on the grid

    lambda_i = -pi + 2 pi i / n   (i = 0..n-1),   theta_j = (j + 1/2) pi / m   (j = 0..m-1),

stored row-major as ``[m, n]`` float64 (theta slow, lambda fast).  It holds no
part of the Poisson method itself.  The only solution-related helper is the
textbook eigen-relation of the continuous Laplace-Beltrami operator on the
unit sphere, ``Delta Y_l^M = -l(l+1) Y_l^M``, which gives the exact solution
of a band-limited problem (used as a closed-form pin).

Coefficients are drawn as c_lM = z / (1 + l)^2 with z ~ N(0, 1), l = 1..L,
in the order l ascending, then M = -l..l, from
``numpy.random.default_rng([cfg, rhs, tag])``; tags: 0 = coefficients of f,
1 = coefficients of an observed field, 2 = noise, 3 = a finite-difference
direction, 4 = grid sizes, 5 = low-rank factors.

Right-hand sides in low-rank form, f(lambda, theta) = sum_j d_j c_j(theta)
r_j(lambda): ``sphere_field_factors`` writes a band-limited field as its
2L + 1 (theta profile, lambda mode) pairs; ``lowrank_factors`` draws
d_j = z_j 2^-j and random trigonometric polynomials of degree <= L with
coefficients z / (1 + l)^2.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "shsynth.c")
_SO = os.path.join(_HERE, "libshsynth.so")
_lock = threading.Lock()
_handle = None

TAG_F, TAG_OBS, TAG_NOISE, TAG_DIR, TAG_SIZES, TAG_LOWRANK = 0, 1, 2, 3, 4, 5


def build(force: bool = False) -> str:
    """Compile the C synthesis routine (gcc, OpenMP) next to this file."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O3", "-mavx2", "-mfma", "-fopenmp", "-fPIC", "-shared",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


def _lib():
    global _handle
    with _lock:
        if _handle is None:
            lib = ctypes.CDLL(build())
            lib.sh_legendre_sums.restype = ctypes.c_int
            lib.sh_legendre_sums.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
            _handle = lib
    return _handle


def n_coeffs(L: int) -> int:
    return (L + 1) * (L + 1) - 1


def degrees(L: int) -> np.ndarray:
    """Degree l of every coefficient slot, in draw order."""
    return np.concatenate([np.full(2 * l + 1, l) for l in range(1, L + 1)]) if L > 0 \
        else np.zeros(0, dtype=np.int64)


def orders(L: int) -> np.ndarray:
    """Order M of every coefficient slot, in draw order."""
    return np.concatenate([np.arange(-l, l + 1) for l in range(1, L + 1)]) if L > 0 \
        else np.zeros(0, dtype=np.int64)


def draw_coeffs(L: int, seed) -> np.ndarray:
    """c_lM = z / (1 + l)^2, z ~ N(0,1), l = 1..L, M = -l..l."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal(n_coeffs(L))
    return z / (1.0 + degrees(L)) ** 2


def laplacian_inverse_coeffs(c: np.ndarray, L: int) -> np.ndarray:
    """Coefficients of the zero-mean u with Delta u = sum c_lM Y_l^M (l >= 1)."""
    l = degrees(L).astype(np.float64)
    return -c / (l * (l + 1.0))


def legendre_sums(m: int, L: int, coeff_sets) -> tuple[np.ndarray, np.ndarray]:
    """A, B of shape [nsets, L+1, m] (see shsynth.c)."""
    cs = np.ascontiguousarray(np.atleast_2d(np.asarray(coeff_sets, dtype=np.float64)))
    if cs.shape[1] != n_coeffs(L):
        raise ValueError("coefficient length does not match L")
    ns = cs.shape[0]
    A = np.empty((ns, L + 1, m), dtype=np.float64)
    B = np.empty((ns, L + 1, m), dtype=np.float64)
    rc = _lib().sh_legendre_sums(m, L, ns, cs.ctypes.data, A.ctypes.data, B.ctypes.data)
    if rc != 0:
        raise RuntimeError("sh_legendre_sums failed (%d)" % rc)
    return A, B


def synth(n: int, m: int, L: int, coeff_sets) -> np.ndarray:
    """Sample sum_lM c_lM Y_l^M on the (lambda, theta) grid -> [nsets, m, n]."""
    if n % 2 or L >= n // 2:
        raise ValueError("need even n and L < n/2 for an alias-free lambda synthesis")
    A, B = legendre_sums(m, L, coeff_sets)
    ns = A.shape[0]
    # f(lambda_i) = sum_M Re((A_M - i B_M) e^{i M lambda_i}), lambda_i = -pi + 2 pi i / n,
    # so e^{i M lambda_i} = (-1)^M e^{2 pi i M i / n}; written as an inverse real DFT.
    H = np.zeros((ns, m, n // 2 + 1), dtype=np.complex128)
    sign = np.where(np.arange(L + 1) % 2 == 0, 1.0, -1.0)
    Hm = (A - 1j * B) * sign[None, :, None]          # [ns, L+1, m]
    H[:, :, : L + 1] = np.transpose(Hm, (0, 2, 1))
    H[:, :, 0] *= n
    H[:, :, 1: L + 1] *= n / 2.0
    return np.fft.irfft(H, n=n, axis=2)


def sphere_field(cfg: int, rhs: int, n: int, m: int, L: int, tag: int = TAG_F,
                 with_solution: bool = False):
    """The seeded band-limited field for (config, rhs, tag); optionally also the
    exact zero-mean solution of Delta u = f."""
    c = draw_coeffs(L, [cfg, rhs, tag])
    if with_solution:
        F = synth(n, m, L, [c, laplacian_inverse_coeffs(c, L)])
        return F[0], F[1]
    return synth(n, m, L, [c])[0]


def noise(cfg: int, rhs: int, shape, std: float) -> np.ndarray:
    rng = np.random.default_rng([cfg, rhs, TAG_NOISE])
    return std * rng.standard_normal(shape)


def direction(cfg: int, rhs: int, shape) -> np.ndarray:
    rng = np.random.default_rng([cfg, rhs, TAG_DIR])
    return rng.standard_normal(shape)


def batch_sizes(cfg: int, count: int, choices) -> np.ndarray:
    """(n_r, m_r) pairs drawn i.i.d. uniformly from `choices` -> [count, 2]."""
    rng = np.random.default_rng([cfg, 0, TAG_SIZES])
    ch = np.asarray(list(choices))
    return ch[rng.integers(0, len(ch), size=(count, 2))]


def grid(n: int, m: int):
    lam = -np.pi + 2.0 * np.pi * np.arange(n) / n
    th = (np.arange(m) + 0.5) * np.pi / m
    return lam, th


def cartesian(n: int, m: int):
    """x, y, z on the grid, each [m, n]."""
    lam, th = grid(n, m)
    L, T = np.meshgrid(lam, th)
    return np.cos(L) * np.sin(T), np.sin(L) * np.sin(T), np.cos(T)


def lowrank_factors(cfg: int, rhs: int, n: int, m: int, K: int, L: int):
    """(d [K], C [K, m], R [K, n]): C[j, t] = c_j(theta_t), R[j, i] = r_j(lambda_i),
    random trigonometric polynomials of degree <= L (cos and sin terms).  The
    product need not be smooth at the poles: these exercise the arithmetic of
    a low-rank right-hand side, not the regularity of a field on the sphere."""
    rng = np.random.default_rng([cfg, rhs, TAG_LOWRANK])
    lam, th = grid(n, m)
    d = rng.standard_normal(K) * 2.0 ** -np.arange(K)
    l = np.arange(L + 1)
    w = 1.0 / (1.0 + l) ** 2
    ac, bc, ar, br = (rng.standard_normal((K, L + 1)) * w for _ in range(4))
    C = ac @ np.cos(np.outer(l, th)) + bc @ np.sin(np.outer(l, th))
    R = ar @ np.cos(np.outer(l, lam)) + br @ np.sin(np.outer(l, lam))
    return d, C, R


def sphere_field_factors(cfg: int, rhs: int, n: int, m: int, L: int, tag: int = TAG_F,
                         with_solution: bool = False):
    """The seeded band-limited field of ``sphere_field`` in low-rank form:
    f = sum_{M=0}^{L} A_M(theta) cos(M lambda) + sum_{M=1}^{L} B_M(theta) sin(M lambda),
    rank K = 2L + 1, d = 1.  Returns (d, C, R) and optionally the exact
    zero-mean solution of Delta u = f on the grid."""
    c = draw_coeffs(L, [cfg, rhs, tag])
    A, B = legendre_sums(m, L, [c])
    lam, _ = grid(n, m)
    M = np.arange(L + 1)
    C = np.vstack([A[0], B[0, 1:]])
    R = np.vstack([np.cos(np.outer(M, lam)), np.sin(np.outer(M[1:], lam))])
    d = np.ones(2 * L + 1)
    if with_solution:
        return d, C, R, synth(n, m, L, [laplacian_inverse_coeffs(c, L)])[0]
    return d, C, R
