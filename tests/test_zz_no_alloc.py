"""The allocation-free entry point sphere_poisson_ge_lowrank_static (its
workspace a static device array of the library) against the entry point
with a caller workspace, sphere_poisson_ge_lowrank: two calls in a row, the
second on a smaller grid (the static array keeps the first call's contents),
each giving exactly the same pivots and terms (the same kernels in the same
order on the same data); its terms also match the oracle's.  Grids whose
workspace exceeds the static array are rejected before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle.ge as OG
import sh_inputs as S

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import paper_1510_08094_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.library()
    return P


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def static_call(P, f, steps, alpha, tol):
    m, n = f.shape
    dev = f.device
    d = torch.empty(2 * steps, dtype=torch.float64, device=dev)
    c = torch.empty((2 * steps, m), dtype=torch.float64, device=dev)
    r = torch.empty((2 * steps, n), dtype=torch.float64, device=dev)
    piv = torch.empty((steps, 2), dtype=torch.int32, device=dev)
    vp = ctypes.c_void_p
    code = P.library().sphere_poisson_ge_lowrank_static(
        n, m, vp(f.data_ptr()), steps, alpha, tol, vp(d.data_ptr()), vp(c.data_ptr()), vp(r.data_ptr()),
        vp(piv.data_ptr()), vp(torch.cuda.current_stream(dev).cuda_stream))
    return code, d, c, r, piv


@pytest.mark.parametrize("order", ["large_then_small"])
def test_static_workspace_matches_caller_workspace(P, order):
    cases = [(256, 200, 20), (64, 33, 8)]     # the second call on a smaller grid
    for n, m, L in cases:
        print("no-alloc ge", n, m, L, flush=True)
        f = gpu(S.sphere_field(21, L, n, m, L))
        steps = 2 * L + 2
        code, d, c, r, piv = static_call(P, f, steps, 0.01, 1e-12)
        assert code == 0
        d2, c2, r2, piv2 = P.ge_lowrank(f, steps, 0.01, 1e-12)
        torch.cuda.synchronize()
        assert torch.equal(piv, piv2)
        assert torch.equal(d, d2) and torch.equal(c, c2) and torch.equal(r, r2)
        # against the oracle, to the bar of the GE parity tests
        fh = f.cpu().numpy()
        do, co, ro, po, eo = OG.ge_lowrank(fh, steps, 0.01, 1e-12)
        assert np.array_equal(piv.cpu().numpy(), po)
        dh, ch, rh = d.cpu().numpy(), c.cpu().numpy(), r.cpu().numpy()
        scale = np.max(np.abs(fh))
        for q in range(2 * steps):
            assert np.max(np.abs(dh[q] * np.outer(ch[q], rh[q]) - do[q] * np.outer(co[q], ro[q]))) <= 1e-11 * scale


def test_static_workspace_rejects_oversize_grids(P):
    n, m = 4096, 2048                               # 64 MiB of residual: above the 40 MiB array
    assert P.library().sphere_poisson_ge_workspace_bytes(n, m) > (40 << 20)
    f = torch.zeros((m, n), dtype=torch.float64, device="cuda")
    code, *_ = static_call(P, f, 2, 0.01, 0.0)
    assert code == 2                                # SP_ERR_UNSUPPORTED_SIZE
    code, *_ = static_call(P, f[:1, :4].contiguous(), 0, 0.01, 0.0)
    assert code == 1                                # steps < 1
