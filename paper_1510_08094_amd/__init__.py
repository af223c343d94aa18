"""Python binding of the MI355X DFS spectral Poisson solver (C ABI in
include/sphere_poisson.h).  Argument marshalling only: every step of the
solve runs in the HIP library; torch provides device memory and the stream.

The solver follows Townsend, Wilber & Wright, Section 5: samples f[j, i] at
theta_j = (j + 1/2) pi / m, lambda_i = -pi + 2 pi i / n (float64, [m, n])
give samples u of the solution of the sin^2-scaled Poisson equation on the
unit sphere with a prescribed integral of u.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # loads the HIP runtime that the library then shares

__all__ = ["SpherePoisson", "SpherePoissonFunction", "SpherePoissonBatch", "solve_batch", "library",
           "LibraryMissing", "SP_FP64", "SP_MIXED", "SP_SYNC_INFO", "SP_AUTOTUNE", "SP_INFO", "SpError",
           "exported_symbols"]

_HERE = os.path.dirname(os.path.abspath(__file__))
# SPHERE_POISSON_LIB selects another build of the same library (the host-sanitizer build of the CPU checks)
LIB_PATH = os.environ.get("SPHERE_POISSON_LIB") or os.path.join(_HERE, "libsphere_poisson.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "sphere_poisson.h")

SP_FP64, SP_MIXED = 0, 1
SP_SYNC_INFO = 0x1
SP_AUTOTUNE = 0x2
SP_INFO = 0x4
_STATUS = {0: "SP_OK", 1: "SP_ERR_INVALID_ARG", 2: "SP_ERR_UNSUPPORTED_SIZE", 3: "SP_ERR_OOM",
           4: "SP_ERR_HIP", 5: "SP_ERR_NOT_CONVERGED", 6: "SP_ERR_ALIAS", 7: "SP_ERR_NO_DEVICE",
           8: "SP_ERR_BAD_PLAN"}


class LibraryMissing(RuntimeError):
    pass


class SpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_STATUS.get(code, "?"), code, msg))
        self.code = code


class SpDesc(ctypes.Structure):
    _fields_ = [("n_lambda", ctypes.c_int), ("m_theta", ctypes.c_int), ("precision", ctypes.c_int),
                ("max_refine", ctypes.c_int), ("tol", ctypes.c_double), ("flags", ctypes.c_uint),
                ("low_k_fp64", ctypes.c_int)]


class SpInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("rel_correction", ctypes.c_double),
                ("f_integral", ctypes.c_double), ("status", ctypes.c_int),
                ("rel_residual", ctypes.c_double), ("est_rel_err", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def exported_symbols() -> list[str]:
    """Function names declared in the C header."""
    with open(HEADER) as fh:
        text = fh.read()
    return re.findall(r"^\s*(?:int|const char\*|size_t)\s+(sphere_poisson_\w+)\s*\(", text, re.M)


def library():
    """Load the in-tree HIP library (raises LibraryMissing if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing("HIP library %s is not built; run `python -m paper_1510_08094_amd.build`"
                             % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, ci, cd = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    lib.sphere_poisson_plan.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(SpDesc), vp]
    lib.sphere_poisson_solve.argtypes = [vp, vp, vp, cd, vp, ctypes.POINTER(SpInfo)]
    lib.sphere_poisson_solve_adjoint.argtypes = [vp, vp, vp, vp, ctypes.POINTER(SpInfo)]
    lib.sphere_poisson_solve_lowrank.argtypes = [vp, ci, vp, vp, vp, vp, cd, vp, ctypes.POINTER(SpInfo)]
    lib.sphere_poisson_eval_lowrank.argtypes = [vp, ci, vp, vp, vp, ci, vp, vp, vp]
    lib.sphere_poisson_ge_workspace_bytes.argtypes = [ci, ci]
    lib.sphere_poisson_ge_workspace_bytes.restype = ctypes.c_size_t
    lib.sphere_poisson_ge_lowrank.argtypes = [ci, ci, vp, ci, cd, cd, vp, ctypes.c_size_t, vp, vp, vp, vp, vp]
    lib.sphere_poisson_ge_lowrank_static.argtypes = [ci, ci, vp, ci, cd, cd, vp, vp, vp, vp, vp]
    lib.sphere_poisson_batch_plan.argtypes = [ctypes.POINTER(vp), ci, ctypes.POINTER(ci), ctypes.POINTER(ci),
                                              ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.POINTER(SpDesc), vp]
    lib.sphere_poisson_solve_batch.argtypes = [vp, vp, ctypes.POINTER(SpInfo)]
    lib.sphere_poisson_batch_destroy.argtypes = [vp]
    lib.sphere_poisson_get_info.argtypes = [vp, vp, ctypes.POINTER(SpInfo)]
    lib.sphere_poisson_stream.argtypes = [ci, vp, vp, ctypes.c_size_t, vp]
    lib.sphere_poisson_stream_partials.argtypes = [ctypes.c_size_t]
    lib.sphere_poisson_stream_partials.restype = ctypes.c_size_t
    lib.sphere_poisson_destroy.argtypes = [vp]
    lib.sphere_poisson_strerror.argtypes = [ci]
    lib.sphere_poisson_strerror.restype = ctypes.c_char_p
    lib.sphere_poisson_workspace_bytes.argtypes = [ctypes.POINTER(SpDesc)]
    lib.sphere_poisson_workspace_bytes.restype = ctypes.c_size_t
    lib.sphere_poisson_transform_roundtrip.argtypes = [vp, vp, vp, vp]
    lib.sphere_poisson_tangential_gradient.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sphere_poisson_curl_scalar.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sphere_poisson_divergence.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sphere_poisson_curl.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp]
    lib.sphere_poisson_vorticity.argtypes = [vp, vp, vp, vp, vp, vp]
    lib.sphere_poisson_integral.argtypes = [vp, vp, vp, vp]
    lib.sphere_poisson_profile_enable.argtypes = [vp, ci]
    lib.sphere_poisson_profile_read.argtypes = [vp, ctypes.POINTER(cd), ctypes.POINTER(ci)]
    for name in ("sphere_poisson_profile_enable", "sphere_poisson_profile_read", "sphere_poisson_plan", "sphere_poisson_solve", "sphere_poisson_solve_adjoint",
                 "sphere_poisson_solve_batch", "sphere_poisson_destroy", "sphere_poisson_batch_plan",
                 "sphere_poisson_batch_destroy", "sphere_poisson_get_info", "sphere_poisson_stream",
                 "sphere_poisson_transform_roundtrip", "sphere_poisson_tangential_gradient",
                 "sphere_poisson_curl_scalar", "sphere_poisson_divergence", "sphere_poisson_curl",
                 "sphere_poisson_vorticity", "sphere_poisson_integral", "sphere_poisson_solve_lowrank",
                 "sphere_poisson_eval_lowrank", "sphere_poisson_ge_lowrank", "sphere_poisson_ge_lowrank_static"):
        getattr(lib, name).restype = ci
    _lib = lib
    return lib


def _check(code: int):
    if code != 0:
        raise SpError(code, library().sphere_poisson_strerror(code).decode())


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_grid(t: torch.Tensor, m: int, n: int, name: str):
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda":
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != torch.float64:
        raise TypeError("%s must be float64" % name)
    if tuple(t.shape) != (m, n):
        raise ValueError("%s must have shape (m, n) = (%d, %d), got %s" % (name, m, n, tuple(t.shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)


class SpherePoisson:
    """A plan for one grid size and precision (owns the device workspace)."""

    def __init__(self, n: int, m: int, precision: str = "fp64", max_refine: int = 1, tol: float = 0.0,
                 sync_info: bool = False, device=None, low_k_fp64: int = -1, autotune: bool = False,
                 collect_info: bool = False):
        lib = library()
        self.n, self.m = int(n), int(m)
        self.precision = {"fp64": SP_FP64, "mixed": SP_MIXED}[precision]
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else
                                   torch.device(device).index or 0)
        self.desc = SpDesc(self.n, self.m, self.precision, int(max_refine), float(tol),
                           (SP_SYNC_INFO if sync_info else 0) | (SP_AUTOTUNE if autotune else 0) |
                           (SP_INFO if collect_info else 0),
                           int(low_k_fp64))
        self._plan = ctypes.c_void_p()
        self.info = SpInfo()
        with torch.cuda.device(self.device):
            _check(lib.sphere_poisson_plan(ctypes.byref(self._plan), ctypes.byref(self.desc),
                                           ctypes.c_void_p(_stream_handle(self.device))))

    def solve(self, f: torch.Tensor, integral: float = 0.0, out: torch.Tensor | None = None) -> torch.Tensor:
        _check_grid(f, self.m, self.n, "f")
        u = torch.empty_like(f) if out is None else out
        _check_grid(u, self.m, self.n, "out")
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_solve(self._plan, ctypes.c_void_p(f.data_ptr()),
                                                  ctypes.c_void_p(u.data_ptr()), float(integral),
                                                  ctypes.c_void_p(_stream_handle(self.device)),
                                                  ctypes.byref(self.info)))
        return u

    def solve_lowrank(self, d: torch.Tensor, c: torch.Tensor, r: torch.Tensor, integral: float = 0.0,
                      out: torch.Tensor | None = None) -> torch.Tensor:
        """Solve for f = sum_q d[q] c[q](theta) r[q](lambda) given as factors:
        d [K], c [K, m] (samples at theta_j), r [K, n] (samples at lambda_i),
        float64 device tensors (Section 3, eq. lowrankRepresentation)."""
        K = d.shape[0] if isinstance(d, torch.Tensor) and d.dim() == 1 else -1
        if K < 1:
            raise ValueError("d must be a 1-D tensor of length rank >= 1")
        _check_grid(c, K, self.m, "c")
        _check_grid(r, K, self.n, "r")
        _check_grid(d.view(1, K), 1, K, "d")
        u = torch.empty((self.m, self.n), dtype=torch.float64, device=c.device) if out is None else out
        _check_grid(u, self.m, self.n, "out")
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_solve_lowrank(
                self._plan, K, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(u.data_ptr()), float(integral),
                ctypes.c_void_p(_stream_handle(self.device)), ctypes.byref(self.info)))
        return u

    def eval_lowrank(self, d: torch.Tensor, c: torch.Tensor, r: torch.Tensor, xyz: torch.Tensor,
                     out: torch.Tensor | None = None) -> torch.Tensor:
        """f at the points xyz [P, 3] (projected radially to the sphere) for f
        given by the factors d [K], c [K, m], r [K, n] on the plan's grid
        (Section 4, Pointwise evaluation)."""
        K = d.shape[0] if isinstance(d, torch.Tensor) and d.dim() == 1 else -1
        if K < 1:
            raise ValueError("d must be a 1-D tensor of length rank >= 1")
        _check_grid(c, K, self.m, "c")
        _check_grid(r, K, self.n, "r")
        _check_grid(d.view(1, K), 1, K, "d")
        if xyz.dim() != 2 or xyz.shape[1] != 3:
            raise ValueError("xyz must have shape (P, 3)")
        P = xyz.shape[0]
        _check_grid(xyz, P, 3, "xyz")
        o = torch.empty(P, dtype=torch.float64, device=xyz.device) if out is None else out
        _check_grid(o.view(1, -1) if o.dim() == 1 else o, 1, P, "out")
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_eval_lowrank(
                self._plan, K, ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(c.data_ptr()),
                ctypes.c_void_p(r.data_ptr()), P, ctypes.c_void_p(xyz.data_ptr()), ctypes.c_void_p(o.data_ptr()),
                ctypes.c_void_p(_stream_handle(self.device))))
        return o

    def adjoint(self, g: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        _check_grid(g, self.m, self.n, "g")
        fb = torch.empty_like(g) if out is None else out
        _check_grid(fb, self.m, self.n, "out")
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_solve_adjoint(self._plan, ctypes.c_void_p(g.data_ptr()),
                                                          ctypes.c_void_p(fb.data_ptr()),
                                                          ctypes.c_void_p(_stream_handle(self.device)),
                                                          ctypes.byref(self.info)))
        return fb

    def get_info(self) -> dict:
        """The info of the last solve or adjoint (synchronises the stream)."""
        info = SpInfo()
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_get_info(self._plan, ctypes.c_void_p(_stream_handle(self.device)),
                                                     ctypes.byref(info)))
        return info.as_dict()

    def roundtrip(self, f: torch.Tensor) -> torch.Tensor:
        _check_grid(f, self.m, self.n, "f")
        out = torch.empty_like(f)
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_transform_roundtrip(
                self._plan, ctypes.c_void_p(f.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                ctypes.c_void_p(_stream_handle(self.device))))
        return out

    def tangential_gradient(self, f: torch.Tensor, outs=None):
        """(d^t f/dx, d^t f/dy, d^t f/dz) on the plan's grid (Section 4, eq.
        diff_x, diff_y, diff_z; float64 whatever the plan's precision)."""
        _check_grid(f, self.m, self.n, "f")
        gs = [torch.empty_like(f) for _ in range(3)] if outs is None else list(outs)
        for g in gs:
            _check_grid(g, self.m, self.n, "out")
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_tangential_gradient(
                self._plan, ctypes.c_void_p(f.data_ptr()), *(ctypes.c_void_p(g.data_ptr()) for g in gs),
                ctypes.c_void_p(_stream_handle(self.device))))
        return tuple(gs)

    def _field_call(self, name, ins, nout, outs):
        for t in ins:
            _check_grid(t, self.m, self.n, "input")
        gs = [torch.empty_like(ins[0]) for _ in range(nout)] if outs is None else list(outs)
        for g in gs:
            _check_grid(g, self.m, self.n, "out")
        with torch.cuda.device(self.device):
            _check(getattr(library(), name)(
                self._plan, *(ctypes.c_void_p(t.data_ptr()) for t in ins),
                *(ctypes.c_void_p(g.data_ptr()) for g in gs), ctypes.c_void_p(_stream_handle(self.device))))
        return tuple(gs) if nout > 1 else gs[0]

    def integral(self, f: torch.Tensor) -> torch.Tensor:
        """Integral of f over the sphere (Section 4, Integration): a 0-d
        float64 tensor on f's device, written asynchronously."""
        _check_grid(f, self.m, self.n, "f")
        out = torch.empty((), dtype=torch.float64, device=f.device)
        with torch.cuda.device(self.device):
            _check(library().sphere_poisson_integral(self._plan, ctypes.c_void_p(f.data_ptr()),
                                                     ctypes.c_void_p(out.data_ptr()),
                                                     ctypes.c_void_p(_stream_handle(self.device))))
        return out

    def curl_scalar(self, f: torch.Tensor, outs=None):
        """n x grad f (Section 4, eq. CurlScalarF): three components."""
        return self._field_call("sphere_poisson_curl_scalar", [f], 3, outs)

    def divergence(self, fx, fy, fz, out=None):
        """Surface divergence of the tangent field (fx, fy, fz)."""
        return self._field_call("sphere_poisson_divergence", [fx, fy, fz], 1, None if out is None else [out])

    def curl(self, fx, fy, fz, outs=None):
        """Surface curl of the tangent field (fx, fy, fz): three components."""
        return self._field_call("sphere_poisson_curl", [fx, fy, fz], 3, outs)

    def vorticity(self, fx, fy, fz, out=None):
        """n . curl of the tangent field (fx, fy, fz)."""
        return self._field_call("sphere_poisson_vorticity", [fx, fy, fz], 1, None if out is None else [out])

    KERNEL_KINDS = ("lambda_fwd", "theta", "lambda_inv", "lambda_mix", "theta_resid", "lambda_upd", "reduce",
                    "lambda_grad", "lowrank", "eval_coeffs", "eval")

    def profile_enable(self, capacity: int):
        """Bracket the next `capacity` kernel launches with HIP events."""
        _check(library().sphere_poisson_profile_enable(self._plan, int(capacity)))

    def profile_read(self) -> dict:
        """{kind: (total_ms, launches)} of the recorded launches (then cleared)."""
        n = len(self.KERNEL_KINDS)
        ms = (ctypes.c_double * n)()
        cnt = (ctypes.c_int * n)()
        _check(library().sphere_poisson_profile_read(self._plan, ms, cnt))
        return {k: (ms[i], cnt[i]) for i, k in enumerate(self.KERNEL_KINDS) if cnt[i]}

    def close(self):
        if self._plan:
            _check(library().sphere_poisson_destroy(self._plan))
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class SpherePoissonFunction(torch.autograd.Function):
    """u = S f with the hand-written adjoint as the backward pass."""

    @staticmethod
    def forward(ctx, f: torch.Tensor, plan: SpherePoisson) -> torch.Tensor:
        ctx.plan = plan
        return plan.solve(f.contiguous())

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        return ctx.plan.adjoint(g.contiguous()), None


def ge_lowrank(f: torch.Tensor, steps: int, alpha: float = 0.01, tol: float = 0.0):
    """Low-rank approximation of the sampled f [m, n] (float64, device) by
    structure-preserving Gaussian elimination (Section 3, Figure
    GaussianElimination): returns (d [2 steps], c [2 steps, m], r [2 steps, n],
    pivots [steps, 2]) with f ~ sum_q d[q] c[q](theta) r[q](lambda), the form
    SpherePoisson.solve_lowrank and eval_lowrank take."""
    if not isinstance(f, torch.Tensor) or f.dim() != 2:
        raise ValueError("f must be a 2-D tensor (m, n)")
    m, n = f.shape
    _check_grid(f, m, n, "f")
    lib = library()
    wb = int(lib.sphere_poisson_ge_workspace_bytes(n, m))
    if wb == 0:
        raise SpError(1, "unsupported grid for the Gaussian elimination")
    dev = f.device
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    d = torch.empty(2 * steps, dtype=torch.float64, device=dev)
    c = torch.empty((2 * steps, m), dtype=torch.float64, device=dev)
    r = torch.empty((2 * steps, n), dtype=torch.float64, device=dev)
    piv = torch.empty((steps, 2), dtype=torch.int32, device=dev)
    with torch.cuda.device(dev):
        _check(lib.sphere_poisson_ge_lowrank(n, m, ctypes.c_void_p(f.data_ptr()), int(steps), float(alpha), float(tol),
                                             ctypes.c_void_p(work.data_ptr()), wb, ctypes.c_void_p(d.data_ptr()),
                                             ctypes.c_void_p(c.data_ptr()), ctypes.c_void_p(r.data_ptr()),
                                             ctypes.c_void_p(piv.data_ptr()), ctypes.c_void_p(_stream_handle(dev))))
    return d, c, r, piv


STREAM_KINDS = {"copy": 0, "read": 1, "write": 2}


def stream(kind: str, x: torch.Tensor | None, y: torch.Tensor, nontemporal: bool = False):
    """The achievable-bandwidth kernels (sphere_poisson_stream): kind "copy"
    (y = x), "read" (y receives per-workgroup partial sums of x) or "write"
    (y = 1), on float64 device tensors."""
    lib = library()
    count = y.numel() if kind != "read" else x.numel()
    code = STREAM_KINDS[kind] | (0x10 if nontemporal else 0)
    dev = y.device
    with torch.cuda.device(dev):
        _check(lib.sphere_poisson_stream(code, ctypes.c_void_p(x.data_ptr() if x is not None else 0),
                                         ctypes.c_void_p(y.data_ptr()), count,
                                         ctypes.c_void_p(_stream_handle(dev))))


class SpherePoissonBatch:
    """A batch plan: the problems fs (list of [m_r, n_r] float64 CUDA tensors)
    and their outputs are bound to it; every solve() is one graph launch."""

    def __init__(self, fs, outs=None, precision: str = "mixed", max_refine: int = 1, tol: float = 0.0,
                 autotune: bool = False):
        lib = library()
        self.count = count = len(fs)
        self.fs = list(fs)
        self.us = [torch.empty_like(f) for f in fs] if outs is None else list(outs)
        for f, u in zip(self.fs, self.us):
            _check_grid(f, f.shape[0], f.shape[1], "f")
            _check_grid(u, f.shape[0], f.shape[1], "out")
        ns = (ctypes.c_int * count)(*[int(f.shape[1]) for f in fs])
        ms = (ctypes.c_int * count)(*[int(f.shape[0]) for f in fs])
        fp = (ctypes.c_void_p * count)(*[f.data_ptr() for f in self.fs])
        up = (ctypes.c_void_p * count)(*[u.data_ptr() for u in self.us])
        desc = SpDesc(0, 0, {"fp64": SP_FP64, "mixed": SP_MIXED}[precision], int(max_refine), float(tol),
                      SP_AUTOTUNE if autotune else 0, -1)
        self.device = self.fs[0].device
        self._plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            _check(lib.sphere_poisson_batch_plan(ctypes.byref(self._plan), count, ns, ms, fp, up, ctypes.byref(desc),
                                                 ctypes.c_void_p(_stream_handle(self.device))))
        self.infos = (SpInfo * count)()

    def solve(self, with_info: bool = False):
        """Launch the graph; returns the outputs (and the per-problem infos)."""
        with torch.cuda.device(self.device):
            code = library().sphere_poisson_solve_batch(self._plan, ctypes.c_void_p(_stream_handle(self.device)),
                                                        self.infos if with_info else None)
        if code != 0 and not (with_info and code == 5):
            _check(code)
        if with_info:
            return self.us, [self.infos[r].as_dict() for r in range(self.count)]
        return self.us

    def close(self):
        if self._plan:
            _check(library().sphere_poisson_batch_destroy(self._plan))
            self._plan = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(fs, precision: str = "mixed", outs=None, max_refine: int = 1):
    """Solve every f in `fs` (list of [m_r, n_r] float64 CUDA tensors) with a
    batch plan built for the call."""
    b = SpherePoissonBatch(fs, outs, precision, max_refine)
    us = b.solve()
    b.close()
    return us
