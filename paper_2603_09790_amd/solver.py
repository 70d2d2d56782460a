"""Python front end of libsspcg: argument marshalling around the C ABI.

Every numerical step runs in the HIP library; this module only moves torch
device tensors (memory and the current stream) across the boundary.  Blocks
of vectors are torch tensors of shape (ncols, ld): row j is column j of the
n x ncols block, and ld >= n is the leading dimension.
"""
from __future__ import annotations

import ctypes
import threading

import torch

from . import _lib as L

__all__ = ["Matrix", "solve", "pcg", "spmv", "mpk", "block_update_gram", "gram_rect", "fgs",
           "xr_update", "csr_value_grad", "diffusion7_assemble", "diffusion7_theta_grad",
           "leading_dim", "stream_triad"]


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _dev(device):
    if device is None:
        return torch.device("cuda", torch.cuda.current_device())
    return torch.device(device)


def leading_dim(n: int) -> int:
    """The leading dimension the solver uses for n-row blocks (n rounded up to 64)."""
    return (n + 63) // 64 * 64


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.float64:
        return L.F64
    if t.dtype == torch.float32:
        return L.F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _on(t: torch.Tensor, device, dtype=None) -> torch.Tensor:
    t = torch.as_tensor(t)
    return t.to(device=device, dtype=dtype or t.dtype).contiguous()


def _bytes(nbytes: int, device) -> torch.Tensor:
    """A device buffer of nbytes (torch's allocations are 256-byte aligned)."""
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Matrix:
    """The library's copy of a CSR matrix on one GPU.

    row_ptr / col / val may be numpy arrays or tensors; they are copied to the
    device and kept alive for the handle's lifetime, as is the tensor `aux`
    that holds the library's layout (its size comes from
    sspcg_matrix_aux_bytes).  ``fp32=True`` also keeps FP32 values, which the
    mixed-precision solve and FP32 kernels need.  A symmetric stencil matrix
    is stored as one triangle unless ``full_storage=True`` (needed to update
    it later with non-symmetric values).

    The handle caches one workspace and one pinned poll buffer for the solves
    made through it; a lock serialises those solves (the C library itself
    lets solves with their own workspace and poll buffer run concurrently).
    """

    def __init__(self, row_ptr, col, val, *, fp32: bool = False, full_storage: bool = False,
                 device=None):
        self.device = _dev(device)
        self.handle = None
        with torch.cuda.device(self.device):
            self.row_ptr = _on(row_ptr, self.device, torch.int32)
            self.col = _on(col, self.device, torch.int32)
            self.val = _on(val, self.device, torch.float64)
            self.n = self.row_ptr.numel() - 1
            self.nnz = self.col.numel()
            self.fp32 = fp32
            flags = (L.MATRIX_FP32 if fp32 else 0) | (L.MATRIX_FULL_STORAGE if full_storage else 0)
            lib = L.lib()
            args = (self.n, self.nnz, _p(self.row_ptr), _p(self.col), _p(self.val), flags)
            scratch = _bytes(lib.sspcg_matrix_scratch_bytes(max(self.n, 1)), self.device)
            need = ctypes.c_size_t()
            L.check(lib.sspcg_matrix_aux_bytes(*args, _p(scratch), scratch.numel(),
                                               _stream(self.device), ctypes.byref(need)),
                    "sspcg_matrix_aux_bytes")
            del scratch
            self.aux = _bytes(need.value, self.device)
            h = ctypes.c_void_p()
            L.check(lib.sspcg_matrix_create(*args, _p(self.aux), self.aux.numel(),
                                            _stream(self.device), ctypes.byref(h)),
                    "sspcg_matrix_create")
        self.handle = h
        self._work = None
        self._poll = None
        self._lock = threading.RLock()
        self.values_tag = None

    @classmethod
    def from_csr(cls, A, **kw) -> "Matrix":
        """From any object with row_ptr, col and val attributes."""
        return cls(A.row_ptr, A.col, A.val, **kw)

    def update_values(self, val: torch.Tensor, tag=None) -> None:
        val = _on(val, self.device, torch.float64)
        if val.numel() != self.nnz:
            raise ValueError("value array has the wrong length")
        with torch.cuda.device(self.device):
            L.check(L.lib().sspcg_matrix_update_values(self.handle, _p(val), _stream(self.device)),
                    "sspcg_matrix_update_values")
        self.val = val
        self.values_tag = tag

    def info(self) -> dict:
        v = [ctypes.c_int64() for _ in range(7)]
        L.check(L.lib().sspcg_matrix_info(self.handle, *[ctypes.byref(t) for t in v]),
                "sspcg_matrix_info")
        keys = ("n", "nnz", "slots", "slices", "shared_slices", "device_bytes", "symmetric")
        return {k: t.value for k, t in zip(keys, v)}

    def workspace(self, nbytes: int) -> torch.Tensor:
        if self._work is None or self._work.numel() < nbytes:
            self._work = None
            self._work = _bytes(nbytes, self.device)
        return self._work

    def poll_buffer(self) -> torch.Tensor:
        """Pinned host buffer the solvers poll the device through."""
        if self._poll is None:
            self._poll = torch.empty(L.POLL_BYTES, dtype=torch.uint8, pin_memory=True)
        return self._poll

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            L.lib().sspcg_matrix_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _params(s, sweeps, interval, tol, precision, gram, max_outer, inner_tol, max_refine,
            check_every, profile=False, sweep_tol=0.0, basis="chebyshev",
            graph=False) -> L.Params:
    p = L.Params()
    L.lib().sspcg_default_params(ctypes.byref(p))
    p.s = int(s)
    p.sweeps = int(sweeps)
    p.lambda_min, p.lambda_max = float(interval[0]), float(interval[1])
    p.tol = float(tol)
    p.max_outer = int(max_outer)
    p.precision = {"fp64": L.FP64, "mixed": L.MIXED}[precision]
    p.inner_tol = float(inner_tol)
    p.max_refine = int(max_refine)
    p.gram = {"fgs": L.GRAM_FGS, "cholesky": L.GRAM_CHOLESKY}[gram]
    p.check_every = int(check_every)
    p.profile = 1 if profile else 0
    p.sweep_tol = float(sweep_tol)
    p.basis = L.BASIS[basis]
    p.use_graph = 1 if graph else 0
    return p


def _result(res: L.Result, st: int) -> dict:
    return dict(status=st, status_name=L.status_string(st), outer_iters=res.outer_iters,
                refinements=res.refinements, inner_iters_total=res.inner_iters_total,
                relres=res.relres, relres_true=res.relres_true, device_ms=res.device_ms)


def solve(A: Matrix, b: torch.Tensor, x0: torch.Tensor | None = None, *, s: int = 4,
          sweeps: int = 2, interval=(0.0, 2.0), tol: float = 1e-8, precision: str = "fp64",
          gram: str = "fgs", max_outer: int = 20000, inner_tol: float = 1e-4,
          max_refine: int = 20, check_every: int = 8, history: bool = False,
          profile: bool = False, sweep_tol: float = 0.0, basis: str = "chebyshev",
          graph: bool = False, out: torch.Tensor | None = None, raise_on_error: bool = True):
    """s-step PCG (Algorithm 1) on A x = b.  Returns (x, info).

    info['history'] (when history=True): per outer iteration
    [relres, eta_alpha, eta_beta, conjugacy defect ||B2 - W beta||_F] (fp64),
    or the true relative residual per refinement (mixed).  info['profile']
    (when profile=True): GPU time and launches per phase, from HIP events
    around every phase.  info['relres_true']: ||b - A x|| / ||b|| of the
    returned x, recomputed in FP64 on the device.
    """
    p = _params(s, sweeps, interval, tol, precision, gram, max_outer, inner_tol, max_refine,
                check_every, profile, sweep_tol, basis, graph)
    dev = A.device
    b = _on(b, dev, torch.float64)
    if out is None:
        x = torch.zeros(A.n, dtype=torch.float64, device=dev) if x0 is None \
            else _on(x0, dev, torch.float64).clone()
    else:
        x = out
        if x0 is not None:
            x.copy_(x0)
        else:
            x.zero_()
    nbytes = ctypes.c_size_t()
    L.check(L.lib().sspcg_workspace_bytes(A.handle, ctypes.byref(p), ctypes.byref(nbytes)),
            "sspcg_workspace_bytes")
    res = L.Result()
    nh = (p.max_refine + 1) if precision == "mixed" else L.HIST_STRIDE * p.max_outer
    hist = (ctypes.c_double * nh)() if history else None
    pr = L.Profile()
    with A._lock, torch.cuda.device(dev):
        work = A.workspace(nbytes.value)
        poll = A.poll_buffer()
        st = L.lib().sspcg_solve(A.handle, _p(b), _p(x), ctypes.byref(p), _p(work),
                                 work.numel(), _p(poll), _stream(dev), ctypes.byref(res), hist,
                                 ctypes.byref(pr))
    if raise_on_error:
        L.check(st, "sspcg_solve", allow=(L.OK, L.NOT_CONVERGED))
    info = _result(res, st)
    if profile:
        info["profile"] = pr.as_dict()
    if history:
        import numpy as np
        h = np.ctypeslib.as_array(hist)
        if precision == "mixed":
            info["history"] = h[:res.refinements + 1].copy()
        else:
            k = L.HIST_STRIDE
            info["history"] = h[:k * res.outer_iters].reshape(-1, k).copy()
    return x, info


def pcg(A: Matrix, b: torch.Tensor, x0: torch.Tensor | None = None, *, tol: float = 1e-8,
        max_iter: int = 100000, check_every: int = 16, history: bool = False,
        raise_on_error: bool = True):
    """Classical Jacobi PCG with the same stop test.  Returns (x, info)."""
    p = _params(1, 1, (0.0, 2.0), tol, "fp64", "fgs", max_iter, 1e-4, 0, check_every)
    dev = A.device
    b = _on(b, dev, torch.float64)
    x = torch.zeros(A.n, dtype=torch.float64, device=dev) if x0 is None \
        else _on(x0, dev, torch.float64).clone()
    nbytes = ctypes.c_size_t()
    L.check(L.lib().sspcg_workspace_bytes(A.handle, ctypes.byref(p), ctypes.byref(nbytes)),
            "sspcg_workspace_bytes")
    res = L.Result()
    hist = (ctypes.c_double * max_iter)() if history else None
    with A._lock, torch.cuda.device(dev):
        work = A.workspace(nbytes.value)
        poll = A.poll_buffer()
        st = L.lib().sspcg_pcg_solve(A.handle, _p(b), _p(x), ctypes.byref(p), _p(work),
                                     work.numel(), _p(poll), _stream(dev), ctypes.byref(res),
                                     hist)
    if raise_on_error:
        L.check(st, "sspcg_pcg_solve", allow=(L.OK, L.NOT_CONVERGED))
    info = _result(res, st)
    if history:
        import numpy as np
        info["history"] = np.ctypeslib.as_array(hist)[:res.outer_iters].copy()
    return x, info


INTERVAL_METHODS = {"lanczos": 0, "power": 1}


def interval(A: Matrix, v0: torch.Tensor, *, method: str = "lanczos", steps: int | None = None,
             rtol: float = 1e-3) -> dict:
    """Basis interval [lambda_min, lambda_max] of M^{-1}A estimated on the device.

    method "lanczos": extreme Ritz values of `steps` (default 20) Lanczos
    steps on D^{-1/2} A D^{-1/2}; "power": lambda_min = 0 and the power
    method's lambda_max, stopping at relative change < rtol or after `steps`
    (default 50) steps.  v0: start vector (n values, any non-zero scaling).
    Returns {"interval": (lo, hi), "steps": steps taken}.
    """
    if method not in INTERVAL_METHODS:
        raise ValueError(f"method must be one of {sorted(INTERVAL_METHODS)}")
    if steps is None:
        steps = 20 if method == "lanczos" else 50
    dev = A.device
    v0 = _on(v0, dev, torch.float64)
    if v0.numel() != A.n:
        raise ValueError("v0 must have n entries")
    nbytes = ctypes.c_size_t()
    L.check(L.lib().sspcg_interval_work_bytes(A.handle, steps, ctypes.byref(nbytes)),
            "sspcg_interval_work_bytes")
    lo, hi, taken = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    with A._lock, torch.cuda.device(dev):
        work = A.workspace(nbytes.value)
        L.check(L.lib().sspcg_interval(A.handle, INTERVAL_METHODS[method], steps, rtol, _p(v0),
                                       _p(work), work.numel(), _stream(dev), ctypes.byref(lo),
                                       ctypes.byref(hi), ctypes.byref(taken)), "sspcg_interval")
    return {"interval": (lo.value, hi.value), "steps": taken.value}


# ------------------------------------------------------------------ kernels

def _kwork(s: int, device) -> torch.Tensor:
    return torch.empty(L.lib().sspcg_kernel_work_bytes(s), dtype=torch.uint8, device=device)


def spmv(A: Matrix, x: torch.Tensor) -> torch.Tensor:
    """y = A x (float64, or float32 values/vectors with FP64 sums)."""
    y = torch.empty_like(x)
    with torch.cuda.device(A.device):
        L.check(L.lib().sspcg_spmv(A.handle, _dtype_code(x), _p(x), _p(y), _stream(A.device)),
                "sspcg_spmv")
    return y


def mpk(A: Matrix, r: torch.Tensor, s: int, interval, ld: int | None = None,
        basis: str = "chebyshev"):
    """Algorithm 2: returns Z (s, ld) and P (s+1, ld)."""
    ld = ld or A.n
    Z = torch.zeros((s, ld), dtype=r.dtype, device=A.device)
    P = torch.zeros((s + 1, ld), dtype=r.dtype, device=A.device)
    with torch.cuda.device(A.device):
        L.check(L.lib().sspcg_mpk(A.handle, _dtype_code(r), _p(r), s, float(interval[0]),
                                  float(interval[1]), L.BASIS[basis], _p(Z), _p(P), ld,
                                  _stream(A.device)),
                "sspcg_mpk")
    return Z, P


def block_update_gram(n: int, Z, Q, AZ, AQ, beta, r):
    """In place Q <- Z + Q beta, AQ <- AZ + AQ beta (beta None: Q <- Z, AQ <- AZ);
    returns W = Q^T AQ (s, s) and b1 = Q^T r (s,), float64."""
    s, ld = Q.shape
    dev = Q.device
    W = torch.empty((s, s), dtype=torch.float64, device=dev)
    b1 = torch.empty(s, dtype=torch.float64, device=dev)
    work = _kwork(s, dev)
    beta = None if beta is None else _on(beta, dev, torch.float64)
    with torch.cuda.device(dev):
        L.check(L.lib().sspcg_block_update_gram(n, s, _dtype_code(Q), _p(Z), _p(Q), _p(AZ), _p(AQ),
                                                _p(beta), _p(r), ld, _p(W), _p(b1), _p(work),
                                                work.numel(), _stream(dev)),
                "sspcg_block_update_gram")
    return W, b1


def gram_rect(n: int, Q, AZ):
    """B2 = -Q^T AZ (s, s) float64."""
    s, ld = Q.shape
    dev = Q.device
    B2 = torch.empty((s, s), dtype=torch.float64, device=dev)
    work = _kwork(s, dev)
    with torch.cuda.device(dev):
        L.check(L.lib().sspcg_gram_rect(n, s, _dtype_code(Q), _p(Q), _p(AZ), ld, _p(B2), _p(work),
                                        work.numel(), _stream(dev)), "sspcg_gram_rect")
    return B2


def fgs(W: torch.Tensor, B: torch.Tensor, sweeps: int, solver: str = "fgs",
        sweep_tol: float = 0.0):
    """FGS (or Cholesky) solve of W X = B on the device.  Returns (X, status)."""
    s = W.shape[0]
    vec = B.dim() == 1
    Bm = B.reshape(s, -1).contiguous()
    X = torch.empty_like(Bm)
    status = torch.zeros(1, dtype=torch.int32, device=W.device)
    with torch.cuda.device(W.device):
        L.check(L.lib().sspcg_fgs(s, Bm.shape[1], _p(W.contiguous()), _p(Bm), sweeps,
                                  float(sweep_tol),
                                  {"fgs": L.GRAM_FGS, "cholesky": L.GRAM_CHOLESKY}[solver],
                                  _p(X), _p(status), _stream(W.device)), "sspcg_fgs")
    return (X.reshape(-1) if vec else X), int(status.item())


def xr_update(A: Matrix, Q, AQ, alpha, x, r, z1=None) -> float:
    """In place x += Q alpha, r -= AQ alpha (and z1 = M^{-1} r); returns ||r||^2."""
    s, ld = Q.shape
    rr = torch.empty(1, dtype=torch.float64, device=A.device)
    work = _kwork(s, A.device)
    with torch.cuda.device(A.device):
        L.check(L.lib().sspcg_xr_update(A.handle, s, _dtype_code(Q), _p(Q), _p(AQ),
                                        _p(_on(alpha, A.device, torch.float64)), ld, _p(x), _p(r),
                                        _p(z1), _p(rr), _p(work), work.numel(),
                                        _stream(A.device)), "sspcg_xr_update")
    return float(rr.item())


def csr_value_grad(A: Matrix, lam: torch.Tensor, x: torch.Tensor) -> torch.Tensor:
    g = torch.empty(A.nnz, dtype=torch.float64, device=A.device)
    with torch.cuda.device(A.device):
        L.check(L.lib().sspcg_csr_value_grad(A.handle, _p(lam), _p(x), _p(g), _stream(A.device)),
                "sspcg_csr_value_grad")
    return g


def diffusion7_assemble(A: Matrix, theta: torch.Tensor) -> torch.Tensor:
    val = torch.empty(A.nnz, dtype=torch.float64, device=A.device)
    with torch.cuda.device(A.device):
        L.check(L.lib().sspcg_diffusion7_assemble(A.handle, _p(theta), _p(val), _stream(A.device)),
                "sspcg_diffusion7_assemble")
    return val


def diffusion7_theta_grad(A: Matrix, theta: torch.Tensor, gval: torch.Tensor) -> torch.Tensor:
    g = torch.empty(A.n, dtype=torch.float64, device=A.device)
    with torch.cuda.device(A.device):
        L.check(L.lib().sspcg_diffusion7_theta_grad(A.handle, _p(theta), _p(gval), _p(g),
                                                    _stream(A.device)),
                "sspcg_diffusion7_theta_grad")
    return g


def stream_triad(a: torch.Tensor, b: torch.Tensor, c: torch.Tensor, q: float) -> None:
    """a = b + q c on float64 device tensors (the achievable-bandwidth
    reference of the measurements; not a step of the method)."""
    for t in (a, b, c):
        if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() != a.numel():
            raise ValueError("a, b, c must be contiguous float64 tensors of one length")
    with torch.cuda.device(a.device):
        L.check(L.lib().sspcg_stream_triad(a.numel(), _p(b), _p(c), float(q), _p(a),
                                           _stream(a.device)), "sspcg_stream_triad")
