"""Python access to the CPU oracle (sspcg_oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the solver package.  It shares no code
with the GPU library; only the seeded inputs of ``sspcg_inputs`` are common.

Blocks of vectors are numpy arrays of shape (ncols, n): row j is column j of
the n x ncols block.  Small matrices are (s, s) / (s, nrhs) row-major arrays.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import tempfile

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sspcg_oracle.c")
_OUT = os.path.join(_HERE, "_build")
_LIB = os.path.join(_OUT, "liboracle.so")

OK, NOT_CONVERGED, ERR_ARG, BREAKDOWN, NONFINITE = 0, 1, -1, -3, -5


class Result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("inner_total", ctypes.c_int32),
                ("relres", ctypes.c_double), ("relres_true", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (OpenMP for row loops, no FMA contraction)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    os.makedirs(_OUT, exist_ok=True)
    fd, tmp = tempfile.mkstemp(suffix=".so", dir=_OUT)
    os.close(fd)
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-std=c99", "-Wall", "-o", tmp, _SRC, "-lm"], check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None
_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I = ctypes.c_int
_D = ctypes.c_double


def lib():
    global _lib
    if _lib is not None:
        return _lib
    # SSPCG_ORACLE_LIB names another build of the same source (the mutation
    # tests load copies with a planted mistake this way).
    L = ctypes.CDLL(os.environ.get("SSPCG_ORACLE_LIB") or build())
    sig = {
        "or_version": (_I, []),
        "or_threads": (_I, []),
        "or_set_threads": (None, [_I]),
        "or_dot": (_D, [_I64, _P, _P]),
        "or_nrm2": (_D, [_I64, _P]),
        "or_spmv": (None, [_I64, _P, _P, _P, _P, _P]),
        "or_spmv_f32": (None, [_I64, _P, _P, _P, _P, _P]),
        "or_diagonal": (_I64, [_I64, _P, _P, _P, _P]),
        "or_mpk": (None, [_I64, _P, _P, _P, _P, _P, _I, _D, _D, _P, _P, _I64]),
        "or_mpk_basis": (None, [_I64, _P, _P, _P, _P, _P, _I, _D, _D, _I, _P, _P, _I64]),
        "or_mpk_f32": (None, [_I64, _P, _P, _P, _P, _P, _I, _D, _D, _P, _P, _I64]),
        "or_gram": (None, [_I64, _I, _P, _P, _P, _I64, _P, _P]),
        "or_gram_f32": (None, [_I64, _I, _P, _P, _P, _I64, _P, _P]),
        "or_gram_rect": (None, [_I64, _I, _P, _P, _I64, _P]),
        "or_gram_rect_f32": (None, [_I64, _I, _P, _P, _I64, _P]),
        "or_fgs": (_I, [_I, _I, _P, _P, _I, _P]),
        "or_fgs_tol": (_I, [_I, _I, _P, _P, _I, _D, _P]),
        "or_chol_solve": (_I, [_I, _I, _P, _P, _P]),
        "or_xr_update": (None, [_I64, _I, _P, _P, _P, _I64, _P, _P]),
        "or_xr_update_f32": (None, [_I64, _I, _P, _P, _P, _I64, _P, _P]),
        "or_block_update": (None, [_I64, _I, _P, _P, _P, _P, _P, _I64]),
        "or_block_update_f32": (None, [_I64, _I, _P, _P, _P, _P, _P, _I64]),
        "or_gram_relres": (_D, [_I, _I, _P, _P, _P]),
        "or_gram_resnorm": (_D, [_I, _I, _P, _P, _P]),
        "or_sspcg": (_I, [_I64, _P, _P, _P, _P, _P, _I, _I, _D, _D, _D, _I, _I, _D, _I, _P, _P]),
        "or_sspcg_perturbed": (_I, [_I64, _P, _P, _P, _P, _P, _I, _I, _D, _D, _D, _I, _I, _D,
                                    _I, ctypes.c_uint64, _P, _P]),
        "or_pcg": (_I, [_I64, _P, _P, _P, _P, _P, _D, _I, _P, _P]),
        "or_inner_sspcg_f32": (_I, [_I64, _P, _P, _P, _P, _P, _P, _I, _I, _D, _D, _D, _I,
                                    _P]),
        "or_sspcg_mixed": (_I, [_I64, _P, _P, _P, _P, _P, _I, _I, _D, _D, _D, _D, _I, _I,
                                _P, _P]),
        "or_diffusion7_assemble": (None, [_I64, _P, _P, _P, _P]),
        "or_csr_value_grad": (None, [_I64, _P, _P, _P, _P, _P]),
        "or_diffusion7_theta_grad": (None, [_I64, _P, _P, _P, _P, _P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _p(a: np.ndarray):
    return a.ctypes.data


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _f32(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float32)


def threads() -> int:
    return lib().or_threads()


def set_threads(k: int) -> None:
    """Threads the oracle's row loops may use from now on (k >= 1)."""
    lib().or_set_threads(int(k))


def dot(a, b) -> float:
    a, b = _f64(a), _f64(b)
    return lib().or_dot(a.size, _p(a), _p(b))


def spmv(A, x) -> np.ndarray:
    x = _f64(x)
    y = np.empty(A.n)
    lib().or_spmv(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(x), _p(y))
    return y


def spmv_f32(A, val32, x32) -> np.ndarray:
    val32, x32 = _f32(val32), _f32(x32)
    y = np.empty(A.n, dtype=np.float32)
    lib().or_spmv_f32(A.n, _p(A.row_ptr), _p(A.col), _p(val32), _p(x32), _p(y))
    return y


def jacobi_inverse(A) -> np.ndarray:
    d = np.empty(A.n)
    bad = lib().or_diagonal(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(d))
    if bad:
        raise ValueError("matrix has a missing or non-positive diagonal entry")
    return 1.0 / d


def mpk(A, dinv, r, s, interval, basis="chebyshev"):
    """Algorithm 2: returns Z (s, n) and P (s+1, n)."""
    dinv, r = _f64(dinv), _f64(r)
    Z = np.empty((s, A.n))
    P = np.empty((s + 1, A.n))
    if basis == "chebyshev":
        lib().or_mpk(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(dinv), _p(r), s,
                     interval[0], interval[1], _p(Z), _p(P), A.n)
    else:
        lib().or_mpk_basis(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(dinv), _p(r), s,
                           interval[0], interval[1], 1, _p(Z), _p(P), A.n)
    return Z, P


def mpk_f32(A, val32, dinv32, r32, s, interval):
    val32, dinv32, r32 = _f32(val32), _f32(dinv32), _f32(r32)
    Z = np.empty((s, A.n), dtype=np.float32)
    P = np.empty((s + 1, A.n), dtype=np.float32)
    lib().or_mpk_f32(A.n, _p(A.row_ptr), _p(A.col), _p(val32), _p(dinv32), _p(r32), s,
                     interval[0], interval[1], _p(Z), _p(P), A.n)
    return Z, P


def gram(Q, AQ, r):
    """W = Q^T AQ (lower triangle mirrored) and b1 = Q^T r."""
    s, n = Q.shape
    W = np.empty((s, s))
    b1 = np.empty(s)
    if Q.dtype == np.float32:
        Q, AQ, r = _f32(Q), _f32(AQ), _f32(r)
        lib().or_gram_f32(n, s, _p(Q), _p(AQ), _p(r), n, _p(W), _p(b1))
    else:
        Q, AQ, r = _f64(Q), _f64(AQ), _f64(r)
        lib().or_gram(n, s, _p(Q), _p(AQ), _p(r), n, _p(W), _p(b1))
    return W, b1


def gram_rect(Q, AZ):
    """B2 = -Q^T AZ."""
    s, n = Q.shape
    B2 = np.empty((s, s))
    if Q.dtype == np.float32:
        Q, AZ = _f32(Q), _f32(AZ)
        lib().or_gram_rect_f32(n, s, _p(Q), _p(AZ), n, _p(B2))
    else:
        Q, AZ = _f64(Q), _f64(AZ)
        lib().or_gram_rect(n, s, _p(Q), _p(AZ), n, _p(B2))
    return B2


def fgs(W, B, sweeps, sweep_tol=0.0):
    """nu FGS sweeps from zero (fewer per column once ||m - W a|| <= sweep_tol
    ||m|| when sweep_tol > 0).  B is (s,) or (s, nrhs).  Returns (X, status)."""
    W = _f64(W)
    vec = np.ndim(B) == 1
    B = _f64(B).reshape(W.shape[0], -1)
    X = np.empty_like(B)
    if sweep_tol > 0.0:
        st = lib().or_fgs_tol(W.shape[0], B.shape[1], _p(W), _p(B), sweeps, sweep_tol, _p(X))
    else:
        st = lib().or_fgs(W.shape[0], B.shape[1], _p(W), _p(B), sweeps, _p(X))
    return (X.reshape(-1) if vec else X), st


def chol_solve(W, B):
    W = _f64(W)
    vec = np.ndim(B) == 1
    B = _f64(B).reshape(W.shape[0], -1)
    X = np.empty_like(B)
    st = lib().or_chol_solve(W.shape[0], B.shape[1], _p(W), _p(B), _p(X))
    return (X.reshape(-1) if vec else X), st


def xr_update(Q, AQ, alpha, x, r):
    """In place: x += Q alpha, r -= AQ alpha (FP64 or FP32 storage)."""
    s, n = Q.shape
    alpha = _f64(alpha)
    f = lib().or_xr_update_f32 if Q.dtype == np.float32 else lib().or_xr_update
    f(n, s, _p(Q), _p(AQ), _p(alpha), n, _p(x), _p(r))


def block_update(Z, Q, AZ, AQ, beta):
    """In place: Q <- Z + Q beta, AQ <- AZ + AQ beta."""
    s, n = Q.shape
    beta = _f64(beta)
    f = lib().or_block_update_f32 if Q.dtype == np.float32 else lib().or_block_update
    f(n, s, _p(Z), _p(Q), _p(AZ), _p(AQ), _p(beta), n)


def gram_relres(W, B, X) -> float:
    W = _f64(W)
    B = _f64(B).reshape(W.shape[0], -1)
    X = _f64(X).reshape(W.shape[0], -1)
    return lib().or_gram_relres(W.shape[0], B.shape[1], _p(W), _p(B), _p(X))


def gram_resnorm(W, B, X) -> float:
    """||B - W X||_F."""
    W = _f64(W)
    B = _f64(B).reshape(W.shape[0], -1)
    X = _f64(X).reshape(W.shape[0], -1)
    return lib().or_gram_resnorm(W.shape[0], B.shape[1], _p(W), _p(B), _p(X))


def sspcg(A, b, x0=None, *, s, sweeps, interval, tol, max_outer=20000,
          gram="fgs", sweep_tol=0.0, basis="chebyshev", history=False, perturb_seed=0):
    """Algorithm 1.  Returns (x, result dict[, history (k, 4)]): per outer
    iteration the relative residual, eta_alpha, eta_beta and the conjugacy
    defect ||B2 - W beta||_F.  perturb_seed != 0 moves every Gram entry one
    unit in the last place (seeded random direction) before it is solved."""
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    hist = np.zeros((max_outer, 4)) if history else None
    res = Result()
    lib().or_sspcg_perturbed(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(b), _p(x), s,
                             sweeps, interval[0], interval[1], tol, max_outer,
                             1 if gram == "cholesky" else 0, sweep_tol,
                             0 if basis == "chebyshev" else 1, int(perturb_seed),
                             None if hist is None else _p(hist), ctypes.byref(res))
    out = res.as_dict()
    if history:
        return x, out, hist[:out["iters"]]
    return x, out


def pcg(A, b, x0=None, *, tol, max_iter=100000, history=False):
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    hist = np.zeros(max_iter) if history else None
    res = Result()
    lib().or_pcg(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(b), _p(x), tol, max_iter,
                 None if hist is None else _p(hist), ctypes.byref(res))
    out = res.as_dict()
    if history:
        return x, out, hist[:out["iters"]]
    return x, out


def sspcg_mixed(A, b, x0=None, *, s, sweeps, interval, tol, inner_tol=1e-4,
                max_inner=20000, max_refine=20, history=False):
    b = _f64(b)
    x = np.zeros(A.n) if x0 is None else _f64(x0).copy()
    hist = np.zeros(max_refine + 1)
    res = Result()
    lib().or_sspcg_mixed(A.n, _p(A.row_ptr), _p(A.col), _p(A.val), _p(b), _p(x), s, sweeps,
                         interval[0], interval[1], tol, inner_tol, max_inner, max_refine,
                         _p(hist), ctypes.byref(res))
    out = res.as_dict()
    if history:
        return x, out, hist[:out["refinements"] + 1]
    return x, out


def inner_sspcg_f32(A, val32, dinv32, r32, *, s, sweeps, interval, inner_tol, max_inner):
    """The refinement's inner solve: FP32-storage s-step PCG for A d = r32
    from d = 0.  Returns (d, status, outer iterations)."""
    val32, dinv32, r32 = _f32(val32), _f32(dinv32), _f32(r32)
    d = np.empty(A.n, dtype=np.float32)
    it = ctypes.c_int(0)
    st = lib().or_inner_sspcg_f32(A.n, _p(A.row_ptr), _p(A.col), _p(val32), _p(dinv32),
                                  _p(r32), _p(d), s, sweeps, interval[0], interval[1],
                                  inner_tol, max_inner, ctypes.byref(it))
    return d, st, it.value


def diffusion7_assemble(A, theta) -> np.ndarray:
    theta = _f64(theta)
    val = np.empty(A.nnz)
    lib().or_diffusion7_assemble(A.n, _p(A.row_ptr), _p(A.col), _p(theta), _p(val))
    return val


def csr_value_grad(A, lam, x) -> np.ndarray:
    lam, x = _f64(lam), _f64(x)
    g = np.empty(A.nnz)
    lib().or_csr_value_grad(A.n, _p(A.row_ptr), _p(A.col), _p(lam), _p(x), _p(g))
    return g


def diffusion7_theta_grad(A, theta, gval) -> np.ndarray:
    theta, gval = _f64(theta), _f64(gval)
    g = np.empty(A.n)
    lib().or_diffusion7_theta_grad(A.n, _p(A.row_ptr), _p(A.col), _p(theta), _p(gval), _p(g))
    return g


def lanczos_bounds(A, v0, m=20):
    """Basis interval from m steps of the Lanczos process.

    The Chebyshev basis is scaled by an interval holding the spectrum of the
    Jacobi-preconditioned operator M^{-1}A (Sec. "The s-step PCG method with
    Chebyshev Krylov basis"); M^{-1}A is similar to C = D^{-1/2} A D^{-1/2},
    which is symmetric, so the process runs on C.  Three-term recurrence from
    v_1 = v0/||v0||, no reorthogonalisation:
        alpha_j = v_j^T C v_j
        w = C v_j - alpha_j v_j - beta_{j-1} v_{j-1},  beta_j = ||w||
        v_{j+1} = w / beta_j        (stop early when beta_j = 0)
    The extreme eigenvalues of the tridiagonal T_k = tridiag(beta, alpha,
    beta) are returned with no safety margin: (lambda_min, lambda_max, k).
    At most min(m, n) steps are taken.
    """
    n = A.n
    dh = np.sqrt(jacobi_inverse(A))
    v = _f64(v0).copy()
    nv = np.sqrt(dot(v, v))
    if not (nv > 0.0 and np.isfinite(nv)):
        raise ValueError("start vector has zero norm or non-finite entries")
    v /= nv
    v_prev = np.zeros(n)
    beta_prev = 0.0
    alphas, betas = [], []
    for _ in range(min(m, n)):
        w = dh * spmv(A, dh * v)
        a = dot(v, w)
        w = w - a * v - beta_prev * v_prev
        alphas.append(a)
        beta = np.sqrt(dot(w, w))
        if beta == 0.0:
            break
        betas.append(beta)
        v_prev, v, beta_prev = v, w / beta, beta
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return float(ev[0]), float(ev[-1]), k


def power_bounds(A, v0, rtol=1e-3, max_iter=50):
    """lambda_min = 0 and the power method's lambda_max of M^{-1}A, M = diag(A).

    Follows Sec. "The s-step PCG method with Chebyshev Krylov basis": one
    SpMV and one Jacobi application per step, stopping once successive
    estimates differ by less than rtol relative to the newer one, or after
    max_iter steps.  The estimate of step l is ||M^{-1} A v_l|| with
    ||v_l|| = 1, and v_{l+1} = M^{-1} A v_l / that norm.
    Returns (0.0, lambda_max, steps, estimates).
    """
    dinv = jacobi_inverse(A)
    v = _f64(v0).copy()
    nv = np.sqrt(dot(v, v))
    if not (nv > 0.0 and np.isfinite(nv)):
        raise ValueError("start vector has zero norm or non-finite entries")
    v /= nv
    lam_old, lam, hist = 0.0, 0.0, []
    for _ in range(max_iter):
        w = dinv * spmv(A, v)
        lam = np.sqrt(dot(w, w))
        hist.append(lam)
        v = w / lam
        if abs(lam - lam_old) < rtol * abs(lam):
            break
        lam_old = lam
    return 0.0, float(lam), len(hist), np.array(hist)
