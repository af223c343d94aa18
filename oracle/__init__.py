"""Plain, slow, double-precision CPU oracle for the double-Fourier-sphere (DFS)
spectral Poisson solver of Townsend, Wilber & Wright, "Computing with
functions in spherical and polar geometries I. The sphere" (Section 5).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link anything in this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.
It shares no code with the GPU path.

Two independent modes are provided (see ``sphere_poisson``):

* ``solve_literal`` follows the paper's construction step by step on the
  doubled grid (DFS doubling, 2D Fourier coefficients, the Sylvester/per-k
  systems built from the paper's coefficient matrices, the bordered k=0
  system with the integration weights, evaluation back on the grid);
* ``solve_reduced`` is the contract the GPU path implements: a real FFT in
  lambda, a cosine (even k) or sine (odd k) transform in theta, two
  tridiagonal systems per wavenumber, the k=0 integral constraint, and the
  inverse transforms.  ``adjoint_reduced`` is the exact transpose of it.

Every function states the passage of the paper it follows and is pinned by
tests in ``tests/test_oracle_pins.py`` to values and identities that do not
come from the oracle itself (the paper's worked integral, the paper's
eigenvalue statement, closed-form solutions, brute-force dense solves).
"""
from .sphere_poisson import *  # noqa: F401,F403
from .calculus import *  # noqa: F401,F403
from .lowrank import *  # noqa: F401,F403
from .evaluate import *  # noqa: F401,F403
from .ge import *  # noqa: F401,F403
