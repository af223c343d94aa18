"""The schedule autotuner: candidates are timed on the GPU, the winners are
cached per transform length, and tuned plans and batches still match the oracle."""
import os
import subprocess
import sys

import numpy as np
import pytest
import torch

import oracle as O
import sh_inputs as S
from conftest import rel2

pytestmark = pytest.mark.gpu

SCRIPT = r"""
import sys, numpy as np, torch
sys.path.insert(0, %r)
import paper_1510_08094_amd as P, oracle as O, sh_inputs as S
def rel(a, b): return float(np.linalg.norm(a - b) / np.linalg.norm(b))
f = S.sphere_field(6, 0, 480, 360, 90)
for prec, tol in (("fp64", 1e-12), ("mixed", 1e-10)):
    plan = P.SpherePoisson(480, 360, prec, autotune=True)
    u = plan.solve(torch.from_numpy(f).cuda()).cpu().numpy()
    assert rel(u, O.solve_reduced(f)) <= tol, prec
    plan.close()
fs = [torch.from_numpy(S.sphere_field(6, r, n, m, min(n, m) // 4)).cuda()
      for r, (n, m) in enumerate([(480, 360), (192, 448), (960, 704)])]
us = P.solve_batch(fs, "mixed")
for r, (fg, u) in enumerate(zip(fs, us)):
    assert rel(u.cpu().numpy(), O.solve_reduced(fg.cpu().numpy())) <= 1e-10, r
print("ok")
"""


def test_autotune_fills_cache_and_stays_correct(tmp_path):
    cache = tmp_path / "tune.txt"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SPHERE_POISSON_TUNE_CACHE=str(cache), SPHERE_POISSON_AUTOTUNE="1")
    r = subprocess.run([sys.executable, "-c", SCRIPT % root], env=env, capture_output=True, text=True,
                       timeout=240)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = cache.read_text().splitlines()
    keys = {" ".join(l.split()[:3]) for l in lines}
    assert "gfx950 lam 480" in keys and "gfx950 lam 960" in keys
    assert any(l.startswith("gfx950 theta 360 1 ") for l in lines)
    assert any(l.startswith("gfx950 theta 360 0 ") for l in lines)
    for l in lines:
        radices = [int(x) for x in l.split()[-1].split(":")[-1].split(",")]
        size = int(l.split()[2])
        # lambda: a DFT of length n/2; theta: length m/2 for even m (one real part
        # per workgroup), m for odd m
        assert int(np.prod(radices)) == (size // 2 if (" lam " in l or size % 2 == 0) else size)
