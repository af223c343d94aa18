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
    us = [host(u) for u in P.solve_batch(fg, precision)]
    for r, (f, u) in enumerate(zip(fs, us)):
        m, n = f.shape
        plan = P.SpherePoisson(n, m, precision)
        single = host(plan.solve(fg[r]))
        plan.close()
        # batch tiles and single-plan workgroups differ in thread counts and
        # spectrum layout (different rounding order, same solution)
        assert rel2(u, single) <= (1e-13 if precision == "fp64" else 1e-12), (r, n, m)
        assert rel2(u, O.solve_reduced(f)) <= tol, (r, n, m)
    # a second call with the same sizes and pointers replays the cached graph
    again = [host(u) for u in P.solve_batch(fg, precision)]
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
