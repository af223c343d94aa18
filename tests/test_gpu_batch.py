"""Heterogeneous batches (one graph launch of persistent stage kernels) against
single-problem solves, the oracle and the closed form."""
import numpy as np
import pytest
import torch

import oracle as O
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu

CHOICES = [64 * j for j in range(2, 33)]


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


# every odd prime radix up to 31 appears (n/2 = 32 j, m = 64 j) plus ragged
# blocks; the two odd m run the complex-line theta tiles (small and large radix
# builds), every even m one real part per tile
SMALL = [(128, 192), (1984, 1216), (704, 832), (1088, 1472), (1856, 2048), (2048, 128), (192, 1984),
         (896, 640), (1344, 1600), (320, 448), (128, 128), (1152, 1728), (256, 195), (192, 217)]


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("mixed", 1e-10)])
def test_batch_matches_single_and_oracle(P, precision, tol):
    fs = []
    for r, (n, m) in enumerate(SMALL):
        L = min(n, m) // 4
        fs.append(S.sphere_field(3, 100 + r, n, m, L) + 1e-4 * S.noise(3, 100 + r, (m, n), 1.0))
    fg = [gpu(f) for f in fs]
    batch = P.SpherePoissonBatch(fg, precision=precision)
    us = [host(u) for u in batch.solve()]
    for r, (f, u) in enumerate(zip(fs, us)):
        m, n = f.shape
        plan = P.SpherePoisson(n, m, precision)
        single = host(plan.solve(fg[r]))
        plan.close()
        # batch tiles and single-plan workgroups differ in thread counts and
        # spectrum layout (different rounding order, same solution)
        assert rel2(u, single) <= (1e-13 if precision == "fp64" else 1e-12), (r, n, m)
        assert rel2(u, O.solve_reduced(f)) <= tol, (r, n, m)
    # a second launch of the same plan replays the graph bitwise
    again = [host(u) for u in batch.solve()]
    batch.close()
    for a, b in zip(us, again):
        assert np.array_equal(a, b)


def test_batch_rejects_bad_input(P):
    f = gpu(np.zeros((64, 64)))
    with pytest.raises(P.SpError) as e:
        P.solve_batch([f], "mixed", outs=[f])
    assert e.value.code == 6
    with pytest.raises(P.SpError) as e:
        P.solve_batch([gpu(np.zeros((64, 2 * 37)))], "fp64")
    assert e.value.code == 2


def test_c3_batch_512(P):
    """512 right-hand sides, n and m drawn uniformly from {128, 192, ..., 2048},
    band limit floor(min(n, m)/4), mixed precision, one graph launch: every
    problem against its closed form, a sample against the oracle."""
    sizes = S.batch_sizes(3, 512, CHOICES)
    fs, exact = [], []
    for r, (n, m) in enumerate(sizes):
        f, u = S.sphere_field(3, r, int(n), int(m), int(min(n, m)) // 4, with_solution=True)
        fs.append(f)
        exact.append(u)
    print("c3 inputs ready", flush=True)
    fg = [gpu(f) for f in fs]
    plan_us = P.solve_batch(fg, "mixed")
    us = [host(u) for u in plan_us]
    errs = [rel2(u, e) for u, e in zip(us, exact)]
    print("c3 worst rel err vs closed form", max(errs), flush=True)
    assert max(errs) <= 1e-10
    for r in range(0, 512, 32):
        assert rel2(us[r], O.solve_reduced(fs[r])) <= 1e-10, r


def test_batch_corrections_and_infos(P):
    """max_refine = 2 runs the correction stages twice in the graph: the
    second correction is smaller than the first, both iterates stay within the
    bar, and the infos report the iterations, the correction, the error
    estimate and the integral of f; tol below the last correction marks a
    problem not converged (the outputs are still written)."""
    sizes = [(128, 192), (256, 195), (192, 128), (320, 448)]
    fs = [S.sphere_field(3, 300 + r, n, m, min(n, m) // 4) for r, (n, m) in enumerate(sizes)]
    fg = [gpu(f) for f in fs]
    b1 = P.SpherePoissonBatch(fg, precision="mixed", max_refine=1)
    u1, i1 = b1.solve(with_info=True)
    u1 = [host(u) for u in u1]
    b1.close()
    b2 = P.SpherePoissonBatch(fg, precision="mixed", max_refine=2)
    u2, i2 = b2.solve(with_info=True)
    u2 = [host(u) for u in u2]
    b2.close()
    for r, f in enumerate(fs):
        ref = O.solve_reduced(f)
        assert rel2(u1[r], ref) <= 1e-10 and rel2(u2[r], ref) <= 1e-10, r
        assert i1[r]["iters"] == 1 and i2[r]["iters"] == 2
        assert i2[r]["rel_correction"] < i1[r]["rel_correction"]
        assert 0.0 < i1[r]["est_rel_err"] < 1e-9
        assert i1[r]["status"] == 0 and i2[r]["status"] == 0
        assert abs(i1[r]["f_integral"]) < 1e-10          # band-limited fields with l >= 1
    bt = P.SpherePoissonBatch(fg, precision="mixed", max_refine=1, tol=1e-30)
    ut, it = bt.solve(with_info=True)
    ut = [host(u) for u in ut]
    bt.close()
    assert all(i["status"] == 5 for i in it)
    for r in range(len(fs)):
        assert np.array_equal(ut[r], u1[r])


def test_batch_plan_allocates_once_and_rejects_cross_aliasing(P):
    """Solves on a batch plan reuse its graph (no new plan per call); an output
    overlapping another problem's input is rejected before any device work."""
    a = gpu(np.zeros((64, 64)))
    b = gpu(np.zeros((64, 64)))
    with pytest.raises(P.SpError) as e:
        P.SpherePoissonBatch([a, b], outs=[torch.empty_like(a), a])
    assert e.value.code == 6
    f = gpu(S.sphere_field(3, 7, 64, 48, 12))
    batch = P.SpherePoissonBatch([f, f], precision="fp64")     # shared inputs are allowed
    u0 = [host(u).copy() for u in batch.solve()]
    u1 = [host(u) for u in batch.solve()]
    batch.close()
    assert np.array_equal(u0[0], u0[1]) and np.array_equal(u1[0], u0[0])
