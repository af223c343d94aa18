"""FP64 oracle of the structure-preserving Gaussian elimination (test infrastructure).

Section 3, Figure GaussianElimination and eq. GEstructurePreservingStepPseudoinverse,
discretised on the sampled grid f[t, i] (theta_t = (t + 1/2) pi / m, lambda_i =
-pi + 2 pi i / n, n even).  The doubled function is never formed: by the BMC
symmetry (eq. BMCsphere) its value at (lambda, -theta) is the sample at
(lambda + pi, theta), i.e. column i + n/2 (mod n) of the same row.

Step k, on the residual e (e = f before the first step):
1. Pivot: over the grid points with lambda_i in [0, pi) (i = n/2 .. n-1) and
   every theta_t, the 2 x 2 pivot matrix M = [[a, b], [b, a]] with
   a = e(lambda_i - pi, theta_t) = e[t, i - n/2] and b = e[t, i] has singular
   values |a + b| and |a - b| (eq. SingularValues); the pivot maximises
   sigma_1 = |a| + |b| (the discrete form of the paper's pivot search; ties
   go to the first point in row-major order).
2. eps = alpha sigma_1; the eps-pseudoinverse (Definition pseudoinverse) of the
   centrosymmetric M keeps 1/(a + b) and 1/(a - b) where |a +- b| > eps:
   M^+ = Q diag(g+, g-) Q^T, Q = [[1, 1], [1, -1]] / sqrt 2.
3. e <- e - [e(lambda* - pi, .), e(lambda*, .)] M^+ [e(., theta*); e(., -theta*)]
   (eq. GEstructurePreservingStepPseudoinverse): with the columns
   C0 = e[:, i* - n/2], C1 = e[:, i*] and the rows R0 = e[t*, :],
   R1[i] = e[t*, i + n/2 mod n], the update is the sum of two rank-1 terms
   d (C0 +- C1)(R0 +- R1) with d = g+- / 2.
The approximation after k steps is f - e, the sum of the terms (eq.
lowrankRepresentation: d_j c_j(theta) r_j(lambda)); the + terms pair with
pi-periodic rows and the - terms with pi-antiperiodic rows (eq.
lowrankRepresentationSplit).  The loop stops after `steps` steps, or earlier
once sigma_1 <= tol times the first step's sigma_1 (later terms get d = 0).
The zero-out step at the poles (eq. ZeroOut) is not applied: the grid has no
pole samples.

TEST INFRASTRUCTURE ONLY: nothing in the product path may import or call it.
It shares no code with the GPU path.
"""
from __future__ import annotations

import numpy as np

__all__ = ["ge_lowrank", "pivot_scores", "pivot_inverse", "reflected_row"]


def pivot_scores(e: np.ndarray) -> np.ndarray:
    """sigma_1 of the pivot matrix at every (theta_t, lambda_i), i >= n/2: [m, n/2]."""
    H = e.shape[1] // 2
    return np.abs(e[:, :H]) + np.abs(e[:, H:])


def pivot_inverse(a: float, b: float, eps: float):
    """(g+, g-) of the eps-pseudoinverse Q diag(g+, g-) Q^T of [[a, b], [b, a]]:
    its singular values are |a + b| and |a - b| (eq. SingularValues), kept
    where they exceed eps (Definition pseudoinverse)."""
    return (1.0 / (a + b) if abs(a + b) > eps else 0.0, 1.0 / (a - b) if abs(a - b) > eps else 0.0)


def reflected_row(row: np.ndarray) -> np.ndarray:
    """e(lambda, -theta*) from the row at theta*: the sample at lambda + pi."""
    return np.roll(row, -(row.shape[0] // 2))


def ge_lowrank(f: np.ndarray, steps: int, alpha: float = 0.01, tol: float = 0.0):
    """Returns (d [2 steps], C [2 steps, m], R [2 steps, n], pivots [steps, 2]
    (t*, i*; -1 once stopped), residual e)."""
    m, n = f.shape
    if n % 2:
        raise ValueError("n must be even")
    H = n // 2
    e = np.array(f, dtype=np.float64)
    d = np.zeros(2 * steps)
    C = np.zeros((2 * steps, m))
    R = np.zeros((2 * steps, n))
    piv = -np.ones((steps, 2), dtype=np.int64)
    s_first = None
    for k in range(steps):
        sc = pivot_scores(e)
        flat = int(np.argmax(sc))                 # first maximum in row-major order
        t, ih = divmod(flat, H)
        i = ih + H
        a, b = e[t, i - H], e[t, i]
        s1 = abs(a) + abs(b)
        if s_first is None:
            s_first = s1
        if s1 == 0.0 or s1 <= tol * s_first:
            break
        eps = alpha * s1
        gp, gm = pivot_inverse(a, b, eps)
        C0, C1 = e[:, i - H].copy(), e[:, i].copy()
        R0 = e[t, :].copy()
        R1 = reflected_row(R0)                    # R1[i] = e[t, i + n/2 mod n]
        C[2 * k], C[2 * k + 1] = C0 + C1, C0 - C1
        R[2 * k], R[2 * k + 1] = R0 + R1, R0 - R1
        d[2 * k], d[2 * k + 1] = 0.5 * gp, 0.5 * gm
        e -= d[2 * k] * np.outer(C[2 * k], R[2 * k]) + d[2 * k + 1] * np.outer(C[2 * k + 1], R[2 * k + 1])
        piv[k] = (t, i)
    return d, C, R, piv, e
