"""Low-rank right-hand side on the GPU (Section 3, eq. lowrankRepresentation;
Section 4, Computation of Fourier coefficients), through the C ABI:
parity with the oracle's low-rank route (the paper's X = A D B^T followed by
the Section 5 solve on coefficients) for band-limited fields given as their
(theta profile, lambda mode) factors, with the grid route's contract for
arbitrary factors, with the closed form, and with the dense GPU solve of the
sampled grid.  Float64 bar: relative 2-norm error <= 1e-12; MIXED 1e-10."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import oracle.lowrank as OL
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOL_MIXED = 1e-10


@pytest.fixture(scope="module")
def P():
    import paper_1510_08094_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.library()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def lowrank(P, n, m, d, C, R, precision="fp64", integral=0.0):
    plan = P.SpherePoisson(n, m, precision)
    try:
        return host(plan.solve_lowrank(gpu(d), gpu(C), gpu(R), integral))
    finally:
        plan.close()


# (n, m, L): rank 2L + 1; ragged row groups (m % 16 != 0) and wavenumber tiles
SMOOTH = [(32, 24, 5), (64, 33, 8), (150, 150, 12), (256, 195, 20), (10000, 40, 15), (40, 10000, 15)]


@pytest.mark.parametrize("n,m,L", SMOOTH)
def test_smooth_field_matches_oracle_route_and_closed_form(P, n, m, L):
    print("lowrank smooth", n, m, L, flush=True)
    d, C, R, u_exact = S.sphere_field_factors(11, L, n, m, L, with_solution=True)
    u = lowrank(P, n, m, d, C, R)
    assert rel2(u, OL.solve_lowrank(d, C, R)) <= TOL64
    assert rel2(u, u_exact) <= TOL64


# (n, m, K): K % 4 != 0 exercises the unrolled loop's tail; K = m the largest rank
GENERAL = [(4, 4, 1), (4, 4, 4), (40, 21, 17), (68, 38, 5), (210, 143, 33), (2048, 128, 16), (128, 2000, 7),
           (62, 31, 31)]


@pytest.mark.parametrize("n,m,K", GENERAL)
def test_general_factors_match_grid_contract(P, n, m, K):
    """Arbitrary factors (lambda-dependent values at the poles): the result is
    the solve of the sampled grid, compared with the oracle's grid route and
    with the GPU's own dense solve."""
    print("lowrank general", n, m, K, flush=True)
    d, C, R = S.lowrank_factors(12, K, n, m, K, max(1, min(m, n // 2) - 1))
    f = OL.lowrank_grid(d, C, R)
    u = lowrank(P, n, m, d, C, R)
    assert rel2(u, O.solve_reduced(f)) <= TOL64
    plan = P.SpherePoisson(n, m, "fp64")
    ud = host(plan.solve(gpu(f)))
    plan.close()
    assert rel2(u, ud) <= TOL64


@pytest.mark.parametrize("n,m,L", [(256, 200, 20), (150, 150, 12), (10000, 40, 15)])
def test_mixed_matches_oracle(P, n, m, L):
    print("lowrank mixed", n, m, L, flush=True)
    d, C, R, u_exact = S.sphere_field_factors(13, L, n, m, L, with_solution=True)
    u = lowrank(P, n, m, d, C, R, precision="mixed")
    assert rel2(u, OL.solve_lowrank(d, C, R)) <= TOL_MIXED
    assert rel2(u, u_exact) <= TOL_MIXED


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("mixed", TOL_MIXED)])
def test_full_size_closed_form_and_dense_solve(P, precision, tol):
    """n = m = 10000 (10^8 DOF) with a rank-25 field: the closed form and the
    dense solve of the same grid (the grid is formed on the GPU for the check)."""
    n = m = 10000
    L = 12
    print("lowrank full size", precision, flush=True)
    d, C, R, u_exact = S.sphere_field_factors(14, 0, n, m, L, with_solution=True)
    dg, Cg, Rg = gpu(d), gpu(C), gpu(R)
    plan = P.SpherePoisson(n, m, precision)
    u = plan.solve_lowrank(dg, Cg, Rg)
    f = (Cg.T * dg[None, :]) @ Rg
    ud = plan.solve(f.contiguous())
    torch.cuda.synchronize()
    err_d = float(torch.linalg.norm(u - ud) / torch.linalg.norm(ud))
    del f, ud
    uh = host(u)
    plan.close()
    assert rel2(uh, u_exact) <= tol
    assert err_d <= tol


@pytest.mark.parametrize("c", [0.0, 2.5])
def test_integral_constraint(P, c):
    n, m, L = 64, 48, 9
    d, C, R, u_exact = S.sphere_field_factors(15, 0, n, m, L, with_solution=True)
    u = lowrank(P, n, m, d, C, R, integral=c)
    assert rel2(u, u_exact + c / (4 * np.pi)) <= TOL64


def test_profile_kinds(P):
    n, m, L = 64, 48, 6
    d, C, R = S.sphere_field_factors(16, 0, n, m, L)
    plan = P.SpherePoisson(n, m, "fp64")
    plan.profile_enable(16)
    plan.solve_lowrank(gpu(d), gpu(C), gpu(R))
    torch.cuda.synchronize()
    rec = plan.profile_read()
    plan.close()
    assert rec["lowrank"][1] == 1 and rec["lambda_fwd"][1] == 1
    assert rec["theta"][1] == 1 and rec["lambda_inv"][1] == 1


def test_errors(P):
    n, m = 32, 24
    lib = P.library()
    plan = P.SpherePoisson(n, m, "fp64")
    d, C, R = S.lowrank_factors(17, 0, n, m, m + 1, 4)
    dg, Cg, Rg = gpu(d), gpu(C), gpu(R)
    u = torch.empty((m, n), dtype=torch.float64, device="cuda")
    h = plan._plan
    vp = ctypes.c_void_p

    def call(rank, dd, cc, rr, uu):
        return lib.sphere_poisson_solve_lowrank(h, rank, vp(dd), vp(cc), vp(rr), vp(uu), 0.0, None, None)

    ptr = (dg.data_ptr(), Cg.data_ptr(), Rg.data_ptr(), u.data_ptr())
    assert call(0, *ptr) == 1
    assert call(m + 1, *ptr) == 1
    assert call(3, ptr[0], None, ptr[2], ptr[3]) == 1
    assert call(3, ptr[0], ptr[1], ptr[2], None) == 1
    big = torch.empty((m, n), dtype=torch.float64, device="cuda")
    assert call(3, ptr[0], ptr[1], big.data_ptr(), big.data_ptr()) == 6
    assert call(3, ptr[0], big.data_ptr() + 8 * n, ptr[2], big.data_ptr()) == 6
    assert call(m, *ptr) == 0
    torch.cuda.synchronize()
    plan.close()
    with pytest.raises(ValueError):
        P.SpherePoisson(n, m, "fp64").solve_lowrank(gpu(np.zeros(0)), gpu(np.zeros((0, m))), gpu(np.zeros((0, n))))


@pytest.mark.parametrize("refine,low_k", [(2, -1), (2, 1), (0, -1)])
def test_mixed_refinement_variants(P, refine, low_k):
    """MIXED with two corrections (the second re-transforms u, never f), with
    float32 elimination everywhere (two corrections needed), and with no
    correction (float32 accuracy): the low-rank call follows the dense call."""
    n, m, L = 256, 200, 20
    d, C, R, u_exact = S.sphere_field_factors(18, L, n, m, L, with_solution=True)
    plan = P.SpherePoisson(n, m, "mixed", max_refine=refine, low_k_fp64=low_k, sync_info=True)
    u = host(plan.solve_lowrank(gpu(d), gpu(C), gpu(R)))
    ud = host(plan.solve(gpu(OL.lowrank_grid(d, C, R))))
    plan.close()
    tol = TOL_MIXED if refine > 0 else 1e-5
    assert rel2(u, u_exact) <= tol
    assert rel2(u, ud) <= tol


def test_eval_with_mixed_plan(P):
    """Evaluation does not depend on the plan's precision (float64 tables)."""
    n, m = 64, 48
    d, C, R = S.lowrank_factors(19, 0, n, m, 6, 10)
    pts = np.random.default_rng(5).standard_normal((300, 3))
    outs = []
    for prec in ("fp64", "mixed"):
        plan = P.SpherePoisson(n, m, prec)
        outs.append(host(plan.eval_lowrank(gpu(d), gpu(C), gpu(R), gpu(pts))))
        plan.close()
    assert rel2(outs[1], outs[0]) <= 1e-14
