"""FP64 oracle of the DFS Poisson solver on the unit sphere (test infrastructure).

Notation follows the paper: lambda is the azimuth, theta the colatitude,
(x, y, z) = (cos(lambda) sin(theta), sin(lambda) sin(theta), cos(theta))
(Section 2.1, co-latitude coordinate transform).  A grid function f has shape
[m, n]: row j is theta_j = (j + 1/2) pi / m, column i is
lambda_i = -pi + 2 pi i / n, with n even.

Readings of the paper taken here:

* The per-wavenumber systems of eq. (linearSystems) are taken with the sign
  that column k of the Sylvester equation (SylvesterSphericalPoisson) implies,
  (L - k^2 I) X_k = F_k, where L = M_sin^2 D_m^2 + M_cos M_sin D_m.
* For k = 0 the row q = 0 is replaced by the integration weights,
  2 pi w^T X_0 = c, where c is the prescribed value of the integral of u
  over the sphere (the paper uses c = 0).
* F is the 2D Fourier coefficient matrix of the samples of sin(theta)^2 f~
  (Section 5): samples are scaled first, then transformed.
* The doubled theta grid is the half-shifted grid
  theta'_j' = (j' - m + 1/2) pi / m, j' = 0..2m-1, which contains the
  original samples (j' >= m) and their reflections (j' < m); the poles are
  never sampled.
* The solution returned is the real part of u~ on the m original rows.
"""
from __future__ import annotations

import numpy as np
import scipy.fft as sfft
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "lambda_grid", "theta_grid", "doubled_theta_grid", "dfs_double",
    "coeffs2", "sample2", "coefficient_operators", "sylvester_operator",
    "integration_weights", "sum2", "solve_literal", "solve_coefficients",
    "cos_analysis", "cos_synthesis", "sin_analysis", "sin_synthesis",
    "reduced_bands", "thomas", "solve_reduced", "adjoint_reduced",
    "dense_operator", "surface_integral",
]


# ----------------------------------------------------------------------------
# Grids and the DFS doubling (Section 2.2)
# ----------------------------------------------------------------------------

def lambda_grid(n: int) -> np.ndarray:
    return -np.pi + 2.0 * np.pi * np.arange(n) / n


def theta_grid(m: int) -> np.ndarray:
    return (np.arange(m) + 0.5) * np.pi / m


def doubled_theta_grid(m: int) -> np.ndarray:
    """theta'_j' = (j' - m + 1/2) pi / m for j' = 0..2m-1 (covers (-pi, pi))."""
    return (np.arange(2 * m) - m + 0.5) * np.pi / m


def dfs_double(f: np.ndarray) -> np.ndarray:
    """DFS doubling, Section 2.2 eq. (BMCsphere): f~(lambda, theta) = f(lambda, theta)
    for theta in (0, pi) and f~(lambda, -theta) = f(lambda + pi, theta)
    (a glide reflection).  Returns [2m, n] on the doubled grid."""
    m, n = f.shape
    if n % 2:
        raise ValueError("the doubling needs lambda + pi on the grid: n must be even")
    out = np.empty((2 * m, n), dtype=f.dtype)
    out[m:] = f
    # row j' < m sits at theta = -theta_{m-1-j'}; lambda_i + pi = lambda_{i + n/2}
    out[:m] = np.roll(f[::-1], -n // 2, axis=1)
    return out


# ----------------------------------------------------------------------------
# 2D Fourier coefficients and sampling (Section 4, "Computation of Fourier
# coefficients", eq. (2DFourierExpansion); inverse = the `sample` operation)
# ----------------------------------------------------------------------------

def _mode_ranges(m2: int, n: int):
    return np.arange(-m2 // 2, m2 // 2), np.arange(-n // 2, n // 2)


def coeffs2(gt: np.ndarray, method: str = "auto") -> np.ndarray:
    """Coefficients X[q, k] (q = -m..m-1 rows, k = -n/2..n/2-1 columns) with
    gt(lambda_i, theta'_j') = sum_{q,k} X[q,k] e^{i q theta'_j'} e^{i k lambda_i}
    on the doubled grid ([2m, n] samples).  ``method='dft'`` evaluates the
    defining sums with explicit exponential matrices; ``'fft'`` uses numpy's
    FFT with the explicit phases of the shifted nodes."""
    m2, n = gt.shape
    m = m2 // 2
    qs, ks = _mode_ranges(m2, n)
    th2 = doubled_theta_grid(m)
    lam = lambda_grid(n)
    if method == "auto":
        method = "dft" if max(m2, n) <= 256 else "fft"
    if method == "dft":
        Eq = np.exp(-1j * np.outer(qs, th2))           # [2m, 2m]
        Ek = np.exp(-1j * np.outer(lam, ks))           # [n, n]
        return (Eq @ gt @ Ek) / (m2 * n)
    if method != "fft":
        raise ValueError(method)
    # theta'_j' = -pi + 2 pi (j' + 1/2)/(2m), lambda_i = -pi + 2 pi i/n
    G = np.fft.fft2(gt) / (m2 * n)                     # indices (q mod 2m, k mod n)
    G = G[np.mod(qs, m2)][:, np.mod(ks, n)]
    phase_q = np.exp(1j * np.pi * qs) * np.exp(-1j * np.pi * qs / m2)
    phase_k = np.exp(1j * np.pi * ks)
    return G * phase_q[:, None] * phase_k[None, :]


def sample2(X: np.ndarray, thetas: np.ndarray, n: int, method: str = "auto") -> np.ndarray:
    """Evaluate sum_{q,k} X[q,k] e^{i q theta} e^{i k lambda_i} at the given
    thetas and the n lambda-points (complex result, [len(thetas), n])."""
    m2 = X.shape[0]
    qs, ks = _mode_ranges(m2, n)
    lam = lambda_grid(n)
    if method == "auto":
        method = "dft" if max(m2, n) <= 256 else "fft"
    if method == "dft":
        return np.exp(1j * np.outer(thetas, qs)) @ X @ np.exp(1j * np.outer(ks, lam))
    # only for the doubled grid's own nodes: use the inverse FFT with phases
    m = m2 // 2
    th2 = doubled_theta_grid(m)
    if not np.allclose(thetas, th2[m:]):
        raise ValueError("fft sampling is implemented for the original rows only")
    Y = X * (np.exp(1j * np.pi * qs) * np.exp(1j * np.pi * qs / m2))[:, None] \
          * np.exp(1j * np.pi * ks)[None, :]
    Z = np.zeros((m2, n), dtype=np.complex128)
    Z[np.ix_(np.mod(qs, m2), np.mod(ks, n))] = Y
    full = np.fft.ifft2(Z) * (m2 * n)
    return full[m:]


# ----------------------------------------------------------------------------
# Coefficient operators (Section 5, and eq. (Msin) of Section 4)
# ----------------------------------------------------------------------------

def coefficient_operators(mp: int, sparse: bool = False):
    """D_m, M_cos, M_sin acting on coefficient vectors indexed q = -mp/2..mp/2-1:
    D_m = diag(i q); M_cos = (1/2)(superdiagonal + subdiagonal);
    M_sin = (i/2)(superdiagonal - subdiagonal).  Truncated (no wrap-around)."""
    q = np.arange(-mp // 2, mp // 2)
    if sparse:
        D = sp.diags(1j * q).tocsr()
        up = sp.eye(mp, k=1, dtype=np.complex128, format="csr")
        dn = sp.eye(mp, k=-1, dtype=np.complex128, format="csr")
    else:
        D = np.diag(1j * q)
        up = np.eye(mp, k=1, dtype=np.complex128)
        dn = np.eye(mp, k=-1, dtype=np.complex128)
    Mcos = 0.5 * (up + dn)
    Msin = 0.5j * (up - dn)
    return D, Mcos, Msin


def sylvester_operator(mp: int, sparse: bool = False):
    """L = M_sin^2 D_m^2 + M_cos M_sin D_m, the left factor of eq.
    (SylvesterSphericalPoisson), as the product of the truncated matrices."""
    D, C, S = coefficient_operators(mp, sparse)
    L = S @ S @ D @ D + C @ S @ D
    return L.tocsr() if sparse else L


def integration_weights(mp: int) -> np.ndarray:
    """w_q = (1 + e^{i pi q}) / (1 - q^2), w_{+-1} = 0, q = -mp/2..mp/2-1
    (Section 4, eq. (integrationCoeffs); also the k = 0 constraint in Section 5)."""
    q = np.arange(-mp // 2, mp // 2).astype(np.float64)
    w = np.zeros(mp)
    ok = np.abs(q) != 1
    w[ok] = (1.0 + np.cos(np.pi * q[ok])) / (1.0 - q[ok] ** 2)
    return w


def sum2(f: np.ndarray) -> float:
    """Integral of f over the sphere via the DFS coefficients: the lambda
    integral keeps the k = 0 column (times 2 pi) and the theta integral
    against sin(theta) uses the weights w (Section 4, "Integration")."""
    m, n = f.shape
    X = coeffs2(dfs_double(f))
    k0 = n // 2                         # column of k = 0
    return float(np.real(2.0 * np.pi * np.dot(integration_weights(2 * m), X[:, k0])))


# ----------------------------------------------------------------------------
# Literal mode: the paper's algorithm on the doubled grid (Section 5)
# ----------------------------------------------------------------------------

def solve_literal(f: np.ndarray, integral: float = 0.0, transform: str = "auto",
                  solver: str = "auto") -> np.ndarray:
    """Poisson on the sphere, Section 5, step by step:
    1. double f (eq. BMCsphere) and scale the samples by sin(theta)^2;
    2. take the 2D Fourier coefficients F (eq. tildeuFourierExpansion);
    3.-4. solve for the coefficients of u (``solve_coefficients``);
    5. evaluate sum X_{qk} e^{iq theta} e^{ik lambda} on the original rows.
    ``solver='dense'`` uses LU on the full matrices, ``'banded'`` a sparse
    direct solve of the same matrices."""
    m, n = f.shape
    th2 = doubled_theta_grid(m)
    bt = np.sin(th2)[:, None] ** 2 * dfs_double(f)
    F = coeffs2(bt, transform)
    X = solve_coefficients(F, integral, solver)
    u = sample2(X, theta_grid(m), n, transform)
    return np.real(u)


def solve_coefficients(F: np.ndarray, integral: float = 0.0, solver: str = "auto") -> np.ndarray:
    """Steps 3-4 of Section 5 on the coefficient matrix F of sin(theta)^2 f~
    ([2m, n], q = -m..m-1 rows, k = -n/2..n/2-1 columns):
    3. for each k != 0 solve (L - k^2 I) X_k = F_k (eq. linearSystems, sign
       as read from the Sylvester equation);
    4. for k = 0 replace row q = 0 by w^T with right-hand side c/(2 pi)
       (eq. pentdiagonalPlusRankOne with a prescribed integral c).
    Returns the coefficient matrix X of u~."""
    mp, n = F.shape
    qs, ks = _mode_ranges(mp, n)
    if solver == "auto":
        solver = "dense" if mp <= 256 else "banded"
    sparse = solver == "banded"
    L = sylvester_operator(mp, sparse=sparse)
    w = integration_weights(mp)
    q0 = mp // 2                         # row index of q = 0
    X = np.zeros_like(F)
    I = sp.eye(mp, format="csr") if sparse else np.eye(mp)
    for ci, k in enumerate(ks):
        A = L - float(k) ** 2 * I
        rhs = F[:, ci].copy()
        if k == 0:
            if sparse:
                A = A.tolil()
                A[q0, :] = w
                A = A.tocsc()
            else:
                A = A.copy()
                A[q0, :] = w
            rhs[q0] = integral / (2.0 * np.pi)
        if sparse:
            X[:, ci] = spla.spsolve(sp.csc_matrix(A), rhs)
        else:
            X[:, ci] = np.linalg.solve(A, rhs)
    return X


# ----------------------------------------------------------------------------
# Reduced mode: the same discrete problem after the lambda real transform and
# the even/odd (BMC) symmetry in theta (Section 3, even-periodic/odd-
# antiperiodic split: column k of the doubled function has parity (-1)^k)
# ----------------------------------------------------------------------------

def cos_analysis(x: np.ndarray) -> np.ndarray:
    """a_q with x_j = sum_{q=0}^{m-1} a_q cos(q theta_j) (axis 0)."""
    m = x.shape[0]
    y = sfft.dct(x, type=2, axis=0)            # y_q = 2 sum_j x_j cos(q theta_j)
    a = y / m
    a[0] *= 0.5
    return a


def cos_synthesis(a: np.ndarray) -> np.ndarray:
    """x_j = sum_{q=0}^{m-1} a_q cos(q theta_j) (axis 0)."""
    m = a.shape[0]
    y = a * m
    y[0] *= 2.0
    return sfft.idct(y, type=2, axis=0)


def sin_analysis(x: np.ndarray) -> np.ndarray:
    """b_q (stored at row q-1) with x_j = sum_{q=1}^{m} b_q sin(q theta_j)."""
    m = x.shape[0]
    y = sfft.dst(x, type=2, axis=0)            # y_{q-1} = 2 sum_j x_j sin(q theta_j)
    b = y / m
    b[m - 1] *= 0.5
    return b


def sin_synthesis(b: np.ndarray) -> np.ndarray:
    m = b.shape[0]
    y = b * m
    y[m - 1] *= 2.0
    return sfft.idst(y, type=2, axis=0)


def reduced_bands(p: np.ndarray, k) -> tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Row p of (L - k^2 I) in a cosine or sine basis: the entries multiplying
    the coefficients of index p-2, p, p+2.  They come from applying
    sin^2 d^2/dtheta^2 + cos sin d/dtheta to e^{i q theta} (the operators of
    Section 5), which gives -q^2/2 on the diagonal and (q^2 +- q)/4 two
    places away; k enters as -k^2 on the diagonal."""
    p = np.asarray(p, dtype=np.float64)
    sub = (p - 2.0) * (p - 1.0) / 4.0
    diag = -p * p / 2.0 - np.asarray(k, dtype=np.float64) ** 2
    sup = (p + 2.0) * (p + 1.0) / 4.0
    return sub, diag, sup


def thomas(sub, diag, sup, rhs):
    """Tridiagonal solve without pivoting (Thomas algorithm) along axis 0;
    sub[0] and sup[-1] are ignored.  Trailing axes of rhs are independent
    systems; sub/diag/sup broadcast against rhs."""
    nrow = rhs.shape[0]
    cp = np.empty(np.broadcast(sup, rhs).shape, dtype=np.result_type(sup, rhs))
    dp = np.empty(np.broadcast(diag, rhs).shape, dtype=np.result_type(diag, rhs))
    den = diag[0]
    cp[0] = sup[0] / den
    dp[0] = rhs[0] / den
    for i in range(1, nrow):
        den = diag[i] - sub[i] * cp[i - 1]
        cp[i] = sup[i] / den
        dp[i] = (rhs[i] - sub[i] * dp[i - 1]) / den
    x = np.empty_like(dp)
    x[-1] = dp[-1]
    for i in range(nrow - 2, -1, -1):
        x[i] = dp[i] - cp[i] * x[i + 1]
    return x


def _class_system(qlo: int, qhi: int, start: int, k):
    """Rows/unknowns q = start, start+2, ... <= qhi of a basis with index range
    [qlo, qhi]; neighbours outside [qlo, qhi] are dropped.  Bands are
    [rows, len(k)]."""
    q = np.arange(start, qhi + 1, 2)
    sub, diag, sup = reduced_bands(q[:, None], np.asarray(k, dtype=np.float64)[None, :])
    sub = np.where((q - 2 >= qlo)[:, None], sub, 0.0)
    sup = np.where((q + 2 <= qhi)[:, None], sup, 0.0)
    return q, sub, diag, sup


def _transpose_bands(sub, sup):
    """Bands of T^T: (T^T)_{i,i-1} = T_{i-1,i} = sup[i-1], (T^T)_{i,i+1} = sub[i+1]."""
    z = np.zeros_like(sub[:1])
    return np.concatenate([z, sup[:-1]]), np.concatenate([sub[1:], z])


def _solve_columns(C: np.ndarray, ks: np.ndarray, sine: bool, integral: float,
                   transpose: bool = False) -> np.ndarray:
    """Solve (L - k^2) a = C[:, col] for every column (one wavenumber k each).
    Cosine basis: q = 0..m-1 stored at row q.  Sine basis: q = 1..m stored at
    row q-1.  Each basis splits into an even-q and an odd-q tridiagonal class.
    For k = 0 (cosine basis only) the row q = 0 is the integral constraint,
    a_0 = c/(4 pi) - sum_{q >= 2 even} a_q / (1 - q^2) (the w-row of the
    bordered k = 0 system written in cosine coefficients, w_{+-1} = 0); the
    original row-0 equation is dropped.  ``transpose`` solves with the
    transposed matrices (the adjoint; the affine constant must then be 0)."""
    m = C.shape[0]
    qlo, qhi = (1, m) if sine else (0, m - 1)
    off = 1 if sine else 0
    out = np.zeros_like(C)
    has0 = (not sine) and ks.size > 0 and ks[0] == 0
    rest = np.arange(1 if has0 else 0, ks.size)
    for parity in (0, 1):
        start = parity if parity >= qlo else parity + 2
        q, sub, diag, sup = _class_system(qlo, qhi, start, ks[rest])
        if q.size and rest.size:
            if transpose:
                sub, sup = _transpose_bands(sub, sup)
            out[np.ix_(q - off, rest)] = thomas(sub, diag, sup, C[np.ix_(q - off, rest)])
    if has0:
        # odd class: an ordinary system with k = 0
        q, sub, diag, sup = _class_system(qlo, qhi, 1, [0.0])
        if q.size:
            if transpose:
                sub, sup = _transpose_bands(sub, sup)
            out[q, 0] = thomas(sub, diag, sup, C[q, :1])[:, 0]
        # even class without row 0 / unknown a_0
        q, sub, diag, sup = _class_system(qlo, qhi, 2, [0.0])
        omega = 1.0 / (1.0 - q.astype(np.float64) ** 2)
        if not transpose:
            ae = thomas(sub, diag, sup, C[q, :1])[:, 0] if q.size else np.zeros(0, C.dtype)
            out[q, 0] = ae
            out[0, 0] = integral / (4.0 * np.pi) - np.dot(omega, ae)
        else:
            # transpose of F -> (a_e = T^-1 F_e, a_0 = -omega^T a_e):
            # F_e = T^-T (abar_e - omega abar_0), F_0 = 0
            if q.size:
                sub, sup = _transpose_bands(sub, sup)
                r = C[q, 0] - omega * C[0, 0]
                out[q, 0] = thomas(sub, diag, sup, r[:, None])[:, 0]
            out[0, 0] = 0.0
    return out


def solve_reduced(f: np.ndarray, integral: float = 0.0) -> np.ndarray:
    """Same discrete problem as ``solve_literal``, in real arithmetic:
    a. b = sin(theta_j)^2 f (Section 5 right-hand side);
    b. lambda: real DFT per row, scaled by 1/n (k = 0..n/2);
    c. theta: cosine coefficients for even k, sine coefficients for odd k
       (the doubled column k has parity (-1)^k in theta, Section 3.2);
    d. per k two tridiagonal systems (even and odd q), no pivoting; k = 0
       with the integral constraint;
    e. inverse theta transforms, inverse real DFT in lambda."""
    m, n = f.shape
    if n % 2:
        raise ValueError("n must be even")
    th = theta_grid(m)
    b = np.sin(th)[:, None] ** 2 * f
    B = np.fft.rfft(b, axis=1) / n                     # [m, n/2+1]
    N = n // 2
    X = np.empty_like(B)
    for parity in (0, 1):
        ks = np.arange(parity, N + 1, 2)
        if ks.size == 0:
            continue
        cols = B[:, ks]
        if parity == 0:
            a = cos_analysis(cols)
            a = _solve_columns(a, ks, sine=False, integral=integral)
            X[:, ks] = cos_synthesis(a)
        else:
            bq = sin_analysis(cols)
            bq = _solve_columns(bq, ks, sine=True, integral=0.0)
            X[:, ks] = sin_synthesis(bq)
    return np.fft.irfft(X * n, n=n, axis=1)


def _rfft_weights(n: int) -> np.ndarray:
    c = np.full(n // 2 + 1, 2.0)
    c[0] = 1.0
    c[-1] = 1.0
    return c


def adjoint_reduced(g: np.ndarray) -> np.ndarray:
    """Euclidean transpose of the linear map f -> solve_reduced(f, 0) on grid
    samples.  Factor by factor, in reverse order:
    inverse real DFT^T = real DFT with weights (1, 2, ..., 2, 1);
    synthesis^T = analysis without the 1/m scalings; solve^T = solve with the
    transposed tridiagonals (k = 0: transposed bordered system);
    analysis^T = synthesis with the analysis scalings; real DFT^T (with its
    1/n) = inverse real DFT with weights (1, 1/2, ..., 1/2, 1); then sin^2."""
    m, n = g.shape
    N = n // 2
    cw = _rfft_weights(n)
    G = np.fft.rfft(g, axis=1) * cw[None, :]
    Z = np.empty_like(G)
    th = theta_grid(m)
    for parity in (0, 1):
        ks = np.arange(parity, N + 1, 2)
        if ks.size == 0:
            continue
        cols = G[:, ks]
        if parity == 0:
            # synthesis matrix Phi_{jq} = cos(q theta_j): Phi^T x = dct/2
            abar = sfft.dct(cols, type=2, axis=0) / 2.0
            abar = _solve_columns(abar, ks, sine=False, integral=0.0, transpose=True)
            # analysis = C Phi^T with C = diag(1/m, 2/m, ...): transpose = Phi C
            scale = np.full(m, 2.0 / m)
            scale[0] = 1.0 / m
            Z[:, ks] = _phi_cos(abar * scale[:, None], th)
        else:
            bbar = sfft.dst(cols, type=2, axis=0) / 2.0
            bbar = _solve_columns(bbar, ks, sine=True, integral=0.0, transpose=True)
            scale = np.full(m, 2.0 / m)
            scale[m - 1] = 1.0 / m
            Z[:, ks] = _phi_sin(bbar * scale[:, None], th)
    # transpose of (x -> rfft(x)/n) is Y -> irfft(Y / cw) (numpy's irfft has the 1/n)
    back = np.fft.irfft(Z / cw[None, :], n=n, axis=1)
    return np.sin(th)[:, None] ** 2 * back


def _phi_cos(a: np.ndarray, th: np.ndarray) -> np.ndarray:
    """sum_q a_q cos(q theta_j) (exactly cos_synthesis)."""
    return cos_synthesis(a)


def _phi_sin(b: np.ndarray, th: np.ndarray) -> np.ndarray:
    return sin_synthesis(b)


# ----------------------------------------------------------------------------
# Brute force helpers for pins
# ----------------------------------------------------------------------------

def dense_operator(n: int, m: int, solve=solve_reduced) -> np.ndarray:
    """Matrix of the linear map f -> solve(f, 0) on [m*n] grid vectors,
    assembled column by column (tiny sizes only)."""
    N = n * m
    S = np.empty((N, N))
    e = np.zeros(N)
    for c in range(N):
        e[:] = 0.0
        e[c] = 1.0
        S[:, c] = solve(e.reshape(m, n), 0.0).ravel()
    return S


def surface_integral(u: np.ndarray) -> float:
    """Integral of a band-limited grid function over the sphere from its DFS
    coefficients (same recipe as ``sum2``)."""
    return sum2(u)
