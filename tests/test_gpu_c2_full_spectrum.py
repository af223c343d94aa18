"""Parity at the full workload size, n = m = 10^4 (10^8 samples), with every
wavenumber populated: f = (band-limited field, l <= 2000) + white noise of
std 1e-3, so every lambda-wavenumber k <= 5000 and every theta coefficient q
carries data at the size where the compiled-in length-5000 transforms, the
per-XCD wavenumber slices and the m = 10^4 partitioned eliminations run.

Each precision is compared with the float64 oracle (reduced mode) in three
ways: the relative 2-norm over all samples; the maximum absolute error of
every row against the solution's maximum (so no row hides behind the norm);
and the error of every lambda-wavenumber (the 2-norm over the rows of the
real DFT of u - u_oracle), which may exceed the tolerance times that
wavenumber's own solution norm only by an equal share of the total budget,
tol ||u|| / sqrt(n/2 + 1) (so no band of wavenumbers hides behind the
others)."""
import numpy as np
import pytest
import torch

import oracle as O
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu

N_GRID = M_GRID = 10000


@pytest.fixture(scope="module")
def P():
    import paper_1510_08094_amd as P
    assert torch.cuda.is_available(), "no GPU"
    P.library()
    return P


@pytest.fixture(scope="module")
def problem():
    print("full-spectrum c2: synthesis", flush=True)
    f = S.sphere_field(2, 0, N_GRID, M_GRID, 2000) + S.noise(2, 0, (M_GRID, N_GRID), 1e-3)
    print("full-spectrum c2: oracle", flush=True)
    u = O.solve_reduced(f)
    spec = np.fft.rfft(u, axis=1)
    return f, u, np.sqrt(np.sum(np.abs(spec) ** 2, axis=0))


def gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def check(u, ref, ref_k, tol, what):
    """The three comparisons of the module docstring."""
    e2 = rel2(u, ref)
    d = u - ref
    row_max = np.max(np.abs(d), axis=1)
    umax = np.max(np.abs(ref))
    err_k = np.sqrt(np.sum(np.abs(np.fft.rfft(d, axis=1)) ** 2, axis=0))
    share = tol * np.linalg.norm(ref) / np.sqrt(ref_k.size)
    worst_k = int(np.argmax(err_k - tol * ref_k))
    print("%s: rel 2-norm %.3e, worst row max-abs / max|u| %.3e (row %d), worst wavenumber %d: %.3e of its norm"
          % (what, e2, row_max.max() / umax, int(np.argmax(row_max)), worst_k,
             err_k[worst_k] / max(ref_k[worst_k], 1e-300)), flush=True)
    assert e2 <= tol, what
    assert np.all(row_max <= 10 * tol * umax), what
    assert np.all(err_k <= tol * ref_k + share), what


def test_fp64_full_spectrum(P, problem):
    f, ref, ref_k = problem
    plan = P.SpherePoisson(N_GRID, M_GRID, "fp64")
    u = host(plan.solve(gpu(f)))
    plan.close()
    check(u, ref, ref_k, 1e-12, "fp64")


@pytest.mark.parametrize("low_k,refine", [(-1, 1), (1, 2)])
def test_mixed_full_spectrum(P, problem, low_k, refine):
    """The default mixed solve (float64 elimination for k < max(16, m/64), one
    correction) and the literal precision split of the spec reading
    (float32 eliminations for every k > 0, two corrections)."""
    f, ref, ref_k = problem
    plan = P.SpherePoisson(N_GRID, M_GRID, "mixed", max_refine=refine, low_k_fp64=low_k, sync_info=True)
    u = host(plan.solve(gpu(f)))
    info = plan.info
    plan.close()
    print("mixed low_k %d refine %d: est_rel_err %.3e rel_residual %.3e" % (low_k, refine, info.est_rel_err,
                                                                             info.rel_residual), flush=True)
    check(u, ref, ref_k, 1e-10, "mixed low_k=%d refine=%d" % (low_k, refine))


def test_fp64_adjoint_full_size(P):
    """The float64 adjoint at 10^8 samples against the oracle's transpose, on a
    random (white) g."""
    g = S.noise(2, 1, (M_GRID, N_GRID), 1.0)
    plan = P.SpherePoisson(N_GRID, M_GRID, "fp64")
    fb = host(plan.adjoint(gpu(g)))
    plan.close()
    print("adjoint: gpu done", flush=True)
    ref = O.adjoint_reduced(g)
    e = rel2(fb, ref)
    print("fp64 adjoint rel 2-norm %.3e" % e, flush=True)
    assert e <= 1e-12
