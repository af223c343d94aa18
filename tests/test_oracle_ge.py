"""Pins of the structure-preserving GE oracle (Section 3, Figure
GaussianElimination, eq. GEstructurePreservingStepPseudoinverse, SingularValues,
Definition pseudoinverse, lowrankRepresentationSplit): the pivot matrix's
singular values, the eps-pseudoinverse against an SVD, one step annihilating
the pivot rows and columns, exact recovery of fields of known rank, the
paper's singular example f = 1, and the even/odd structure of the terms."""
import json
import os

import numpy as np
import pytest

import oracle.ge as OG
import sh_inputs as S


def test_singular_values_of_the_pivot_matrix():
    rng = np.random.default_rng(1)
    for a, b in rng.standard_normal((20, 2)):
        sv = np.linalg.svd(np.array([[a, b], [b, a]]), compute_uv=False)
        assert abs(sv[0] - max(abs(a + b), abs(a - b))) <= 1e-14
        assert abs(sv[1] - min(abs(a + b), abs(a - b))) <= 1e-14
        assert abs(sv[0] - (abs(a) + abs(b))) <= 1e-14


@pytest.mark.parametrize("alpha", [0.0, 0.01, 0.5, 0.99])
def test_pseudoinverse_against_svd(alpha):
    rng = np.random.default_rng(2)
    extra = [(1.0, 1.0 + 1e-9)] + ([(1.0, 1.0), (2.0, -2.0)] if alpha > 0 else [])   # exactly singular: the SVD
    for a, b in list(rng.standard_normal((20, 2))) + extra:                       # returns ~1e-16, not 0
        M = np.array([[a, b], [b, a]])
        U, s, Vt = np.linalg.svd(M)
        eps = alpha * s[0]
        sinv = np.array([1.0 / x if x > eps else 0.0 for x in s])
        ref = Vt.T @ np.diag(sinv) @ U.T
        gp, gm = OG.pivot_inverse(a, b, eps)
        got = 0.5 * np.array([[gp + gm, gp - gm], [gp - gm, gp + gm]])
        cond = s[0] / s[1] if s[1] > eps else 1.0          # the SVD's own error grows with it
        assert np.max(np.abs(got - ref)) <= 1e-14 * cond * max(1.0, np.max(np.abs(ref)))


@pytest.mark.parametrize("m,n", [(6, 8), (9, 10), (24, 32)])
def test_one_step_annihilates_pivot_rows_and_columns(m, n):
    """With an invertible pivot (alpha = 0) the residual vanishes on the two
    pivot columns (lambda*, lambda* - pi) and on the pivot row (theta* and its
    reflection -theta*, i.e. the whole sampled row)."""
    f = np.random.default_rng(m * n).standard_normal((m, n))
    d, C, R, piv, e = OG.ge_lowrank(f, 1, alpha=0.0)
    t, i = piv[0]
    H = n // 2
    sc = 1e-13 * np.max(np.abs(f))
    assert np.max(np.abs(e[:, i])) <= sc and np.max(np.abs(e[:, i - H])) <= sc
    assert np.max(np.abs(e[t, :])) <= sc
    assert np.max(np.abs(OG.pivot_scores(f))) == OG.pivot_scores(f)[t, i - H]


@pytest.mark.parametrize("L,m,n", [(3, 12, 16), (5, 24, 32), (10, 64, 48), (12, 150, 150)])
def test_recovers_fields_of_known_rank(L, m, n):
    """A band-limited field of degree L has rank 2L + 1 in (theta, lambda):
    L + 2 steps leave a residual at the rounding level, and the terms sum to
    the approximation f - e."""
    f = S.sphere_field(4, L, n, m, L)
    d, C, R, piv, e = OG.ge_lowrank(f, L + 2, alpha=0.01, tol=1e-12)
    assert np.max(np.abs(e)) <= 1e-13 * np.max(np.abs(f))
    assert np.max(np.abs((C.T * d) @ R - (f - e))) <= 1e-14 * np.max(np.abs(f))
    assert np.count_nonzero(d) <= 2 * L + 2


def test_paper_singular_example_ones():
    """f = 1: every pivot matrix is the all-ones matrix, singular; the
    pseudoinverse keeps 1/(a + b) and one step removes the function."""
    d, C, R, piv, e = OG.ge_lowrank(np.ones((8, 12)), 3)
    assert np.max(np.abs(e)) == 0.0
    assert d[0] == 0.25 and d[1] == 0.0 and np.all(d[2:] == 0)
    assert tuple(piv[0]) == (0, 6) and tuple(piv[1]) == (-1, -1)


def test_terms_have_the_bmc_parity():
    """+ terms pair with pi-periodic rows, - terms with pi-antiperiodic rows."""
    f = S.sphere_field(5, 6, 32, 24, 6)
    d, C, R, piv, e = OG.ge_lowrank(f, 5)
    H = 16
    assert np.max(np.abs(R[0::2, :H] - R[0::2, H:])) <= 1e-15 * np.max(np.abs(R))
    assert np.max(np.abs(R[1::2, :H] + R[1::2, H:])) <= 1e-15 * np.max(np.abs(R))


def test_planted_swapped_pseudoinverse(monkeypatch):
    orig = OG.pivot_inverse
    monkeypatch.setattr(OG, "pivot_inverse", lambda a, b, eps: orig(a, b, eps)[::-1])
    f = np.random.default_rng(7).standard_normal((9, 10))
    d, C, R, piv, e = OG.ge_lowrank(f, 1, alpha=0.0)
    assert np.max(np.abs(e[piv[0][0], :])) > 1e-3


def test_planted_unreflected_row(monkeypatch):
    monkeypatch.setattr(OG, "reflected_row", lambda row: row.copy())
    f = np.random.default_rng(8).standard_normal((9, 10))
    d, C, R, piv, e = OG.ge_lowrank(f, 1, alpha=0.0)
    t, i = piv[0]
    assert max(np.max(np.abs(e[:, i])), np.max(np.abs(e[:, i - 5]))) > 1e-3


GE_TOL = 5e-13   # the stopping tolerance of the numerical-rank reading (golden files)


def _golden(name):
    return json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))


def _paper_field(g):
    x, y, z = S.cartesian(g["n_lambda"], g["m_theta"])
    if g["paper_printed_rank"] == 12:
        return np.sin(50 * x * y * z)
    return np.cos(1 + 2 * np.pi * (x + y) + 5 * np.sin(np.pi * z))


@pytest.mark.parametrize("name", ["sin50xyz_rank.json", "sphere_test_func_rank.json"])
def test_paper_printed_ranks(name):
    """Both numerical ranks the paper prints: 12 for sin(50xyz) (Section 5's
    Poisson example) and 23 for eq. sphereTestFunc (Section 1), on the grid of
    the Poisson example (150 lambda nodes, 75 theta nodes); the golden files
    hold the citations.  The GE stops with the printed number of terms and a
    residual at the rounding level."""
    g = _golden(name)
    f = _paper_field(g)
    d, C, R, piv, e = OG.ge_lowrank(f, 40, alpha=0.01, tol=GE_TOL)
    assert np.count_nonzero(d) == g["paper_printed_rank"]
    assert np.max(np.abs(e)) <= 1e-12 * np.max(np.abs(f))
    if "paper_printed_vertical_scale" in g:
        assert round(float(np.max(np.abs(f)))) == g["paper_printed_vertical_scale"]


@pytest.mark.parametrize("tol", [3e-13, 1e-12])
def test_printed_ranks_hold_across_the_tolerance_window(tol):
    """The reading does not hang on one tolerance: both printed ranks hold at
    the ends of the window around GE_TOL as well."""
    for name in ("sin50xyz_rank.json", "sphere_test_func_rank.json"):
        g = _golden(name)
        d, C, R, piv, e = OG.ge_lowrank(_paper_field(g), 40, alpha=0.01, tol=tol)
        assert np.count_nonzero(d) == g["paper_printed_rank"]


def test_rank_23_needs_a_one_term_step():
    """23 is odd, so at least one step keeps a single term: the
    eps-pseudoinverse (Definition pseudoinverse, eps = alpha sigma_1) drops the
    smaller singular value there.  Without the pseudoinverse (alpha = 0) every
    step adds two terms and the count is even."""
    g = _golden("sphere_test_func_rank.json")
    f = _paper_field(g)
    d, C, R, piv, e = OG.ge_lowrank(f, 40, alpha=0.01, tol=GE_TOL)
    pairs = d.reshape(-1, 2)
    steps = int(np.sum(piv[:, 0] >= 0))
    assert np.any(np.count_nonzero(pairs[:steps], axis=1) == 1)
    d0, *_ = OG.ge_lowrank(f, 40, alpha=0.0, tol=GE_TOL)
    assert np.count_nonzero(d0) % 2 == 0
