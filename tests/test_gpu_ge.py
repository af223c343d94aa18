"""Structure-preserving Gaussian elimination on the GPU (Section 3, Figure
GaussianElimination), through the C ABI: the pivot sequence (an integer
decision, taken in float64 on both sides) equals the oracle's, the terms
match the oracle's within the float64 bar, fields of known rank are
recovered, and the terms feed the low-rank solve and evaluation."""
import ctypes
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import oracle.ge as OG
import oracle.lowrank as OL
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1510_08094_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.library()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def run(P, f, steps, alpha=0.01, tol=0.0):
    d, c, r, piv = P.ge_lowrank(gpu(f), steps, alpha, tol)
    torch.cuda.synchronize()
    return d.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy(), piv.cpu().numpy()


# (n, m, L): a band-limited field of rank 2L + 1; ragged sizes, both n/4 parities
SMOOTH = [(32, 24, 5), (64, 33, 8), (150, 150, 12), (256, 200, 20), (1000, 40, 15), (40, 1000, 15)]


@pytest.mark.parametrize("n,m,L", SMOOTH)
def test_matches_oracle_and_recovers_rank(P, n, m, L):
    print("ge", n, m, L, flush=True)
    f = S.sphere_field(21, L, n, m, L)
    steps = 2 * L + 2
    d, c, r, piv = run(P, f, steps, 0.01, 1e-12)
    do, co, ro, po, eo = OG.ge_lowrank(f, steps, 0.01, 1e-12)
    assert np.array_equal(piv, po)
    scale = np.max(np.abs(f))
    for q in range(2 * steps):
        term = d[q] * np.outer(c[q], r[q])
        ref = do[q] * np.outer(co[q], ro[q])
        assert np.max(np.abs(term - ref)) <= 1e-11 * scale
    rec = OL.lowrank_grid(d, c, r)
    assert np.max(np.abs(rec - f)) <= 1e-12 * scale


def test_paper_singular_example_ones(P):
    d, c, r, piv = run(P, np.ones((8, 12)), 3)
    assert d[0] == 0.25 and np.all(d[1:] == 0)
    assert tuple(piv[0]) == (0, 6) and np.all(piv[1:] == -1)
    assert np.max(np.abs(OL.lowrank_grid(d, c, r) - 1.0)) == 0.0


@pytest.mark.parametrize("n,m", [(10, 9), (64, 48)])
def test_random_grid_first_steps(P, n, m):
    """Random samples (distinct scores): the first steps pick the oracle's
    pivots and terms; the approximation error after them equals the oracle's."""
    f = np.random.default_rng(n + m).standard_normal((m, n))
    steps = 3
    d, c, r, piv = run(P, f, steps, 0.01)
    do, co, ro, po, eo = OG.ge_lowrank(f, steps, 0.01)
    assert np.array_equal(piv, po)
    assert rel2(OL.lowrank_grid(d, c, r), OL.lowrank_grid(do, co, ro)) <= 1e-13


def test_terms_drive_the_lowrank_solve_and_evaluation(P):
    """f -> GE terms -> low-rank solve equals the dense solve of f; the terms
    evaluated at the grid nodes reproduce f."""
    n = m = 150
    L = 12
    f = S.sphere_field(22, 0, n, m, L)
    fg = gpu(f)
    d, c, r, piv = P.ge_lowrank(fg, 2 * L + 2, 0.01, 1e-12)
    plan = P.SpherePoisson(n, m, "fp64")
    u_lr = plan.solve_lowrank(d, c, r)
    u = plan.solve(fg)
    x, y, z = S.cartesian(n, m)
    pts = gpu(np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1))
    fe = plan.eval_lowrank(d, c, r, pts)
    torch.cuda.synchronize()
    plan.close()
    assert rel2(u_lr.cpu().numpy(), u.cpu().numpy()) <= 1e-11
    assert rel2(fe.cpu().numpy().reshape(m, n), f) <= 1e-12


def test_full_size_grid(P):
    """n = m = 10000: a rank-25 field in 14 steps; pivots as the oracle's
    (run on the same samples), reconstruction on sampled rows."""
    n = m = 10000
    L = 12
    f = S.sphere_field(23, 0, n, m, L)
    d, c, r, piv = run(P, f, 2 * L + 2, 0.01, 1e-12)
    rows = np.arange(0, m, 97)
    rec = (c[:, rows].T * d) @ r
    assert np.max(np.abs(rec - f[rows])) <= 1e-12 * np.max(np.abs(f))
    assert np.count_nonzero(d) <= 2 * L + 2


def test_errors(P):
    lib = P.library()
    n, m = 16, 12
    f = gpu(np.ones((m, n)))
    wb = int(lib.sphere_poisson_ge_workspace_bytes(n, m))
    assert wb >= n * m * 8 and lib.sphere_poisson_ge_workspace_bytes(15, m) == 0
    work = torch.empty(wb, dtype=torch.uint8, device="cuda")
    d = torch.empty(4, dtype=torch.float64, device="cuda")
    c = torch.empty((4, m), dtype=torch.float64, device="cuda")
    r = torch.empty((4, n), dtype=torch.float64, device="cuda")
    vp = ctypes.c_void_p

    def call(steps=2, alpha=0.01, tol=0.0, wbytes=wb, rr=None, cc=None):
        return lib.sphere_poisson_ge_lowrank(n, m, vp(f.data_ptr()), steps, alpha, tol, vp(work.data_ptr()), wbytes,
                                             vp(d.data_ptr()), vp(c.data_ptr() if cc is None else cc),
                                             vp(r.data_ptr() if rr is None else rr), None, None)

    assert call(steps=0) == 1
    assert call(alpha=1.5) == 1 and call(alpha=-0.1) == 1 and call(tol=-1.0) == 1
    assert call(wbytes=wb - 1) == 1
    assert call(rr=r.data_ptr() + 8) == 1                      # misaligned rows
    assert call(cc=f.data_ptr()) == 6                          # output over the input
    assert call(rr=work.data_ptr()) == 6                       # output over the workspace
    assert call() == 0
    torch.cuda.synchronize()


@pytest.mark.parametrize("name", ["sin50xyz_rank.json", "sphere_test_func_rank.json"])
def test_paper_printed_ranks_and_poisson(P, name):
    """The paper's two printed numerical ranks on the grid of its Poisson
    example (150 lambda nodes, 75 theta nodes): 12 for sin(50xyz) (Section 5)
    and 23 for eq. sphereTestFunc (Section 1); tests/golden holds the
    citations and the stopping tolerance.  The low-rank solve of the terms
    equals the oracle's solve of the samples (eq. sphereTestFunc has a
    non-zero mean: both sides solve the bordered system as it stands).  Symmetric points of these
    functions can tie in exact arithmetic, so the pivot order is not compared
    (either choice is valid)."""
    g = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))
    m, n = g["m_theta"], g["n_lambda"]
    x, y, z = S.cartesian(n, m)
    if g["paper_printed_rank"] == 12:
        f = np.sin(50 * x * y * z)
    else:
        f = np.cos(1 + 2 * np.pi * (x + y) + 5 * np.sin(np.pi * z))
    d, c, r, piv = P.ge_lowrank(gpu(f), 30, 0.01, 5e-13)   # 60 terms at most: the solve takes rank <= m
    dh = d.cpu().numpy()
    assert np.count_nonzero(dh) == g["paper_printed_rank"]
    rec = OL.lowrank_grid(dh, c.cpu().numpy(), r.cpu().numpy())
    assert np.max(np.abs(rec - f)) <= 1e-12 * np.max(np.abs(f))
    plan = P.SpherePoisson(n, m, "fp64")
    u = plan.solve_lowrank(d, c, r)
    torch.cuda.synchronize()
    uh = u.cpu().numpy()
    plan.close()
    assert rel2(uh, O.solve_reduced(f)) <= 1e-12
