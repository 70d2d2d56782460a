"""sspcg_solve_static (workspace in a static device array, no allocation)
against sspcg_solve (caller's workspace), through the C ABI.

The two entry points run the same kernels on the same inputs with the same
workspace layout, so their results agree bit for bit.  The caller workspace
of sspcg_solve is filled with NaN bit patterns first, and the static array
keeps whatever the previous call left, so an agreement also shows that no
solve reads workspace memory it has not written.
"""
import ctypes

import numpy as np
import pytest
import torch

import paper_2603_09790_amd as P
import sspcg_inputs as si
from paper_2603_09790_amd import _lib as L

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def params(interval, s, sweeps, tol, precision=L.FP64):
    p = L.Params()
    L.lib().sspcg_default_params(ctypes.byref(p))
    p.s, p.sweeps = s, sweeps
    p.lambda_min, p.lambda_max = float(interval[0]), float(interval[1])
    p.tol = tol
    p.precision = precision
    return p


def poll_buffer():
    return torch.empty(L.POLL_BYTES, dtype=torch.uint8, pin_memory=True)


def solve_with_workspace(M, b, p):
    x = torch.zeros(M.n, dtype=torch.float64, device=DEV)
    nbytes = ctypes.c_size_t()
    assert L.lib().sspcg_workspace_bytes(M.handle, ctypes.byref(p), ctypes.byref(nbytes)) == L.OK
    work = torch.full((nbytes.value,), 0xFF, dtype=torch.uint8, device=DEV)   # NaN patterns
    res = L.Result()
    st = L.lib().sspcg_solve(M.handle, _p(b), _p(x), ctypes.byref(p), _p(work), nbytes.value,
                             _p(poll_buffer()), _stream(), ctypes.byref(res), None, None)
    return st, x, res, nbytes.value


def solve_static(M, b, p):
    x = torch.zeros(M.n, dtype=torch.float64, device=DEV)
    res = L.Result()
    st = L.lib().sspcg_solve_static(M.handle, _p(b), _p(x), ctypes.byref(p), _p(poll_buffer()),
                                    _stream(), ctypes.byref(res))
    return st, x, res


CASES = [   # (workload, N, s, sweeps, precision): the second call has a smaller input
    ("poisson7", 40, 4, 2, L.FP64),
    ("poisson5", 24, 6, 2, L.FP64),
    ("diffusion27", 16, 6, 2, L.MIXED),
    ("poisson5", 9, 3, 1, L.FP64),
]


def test_static_solve_matches_workspace_solve():
    for name, N, s, nu, prec in CASES:
        print(f"[static] {name} N={N} s={s} nu={nu} precision={prec}", flush=True)
        w = si.workload(name, N=N)
        M = P.Matrix.from_csr(w["A"], fp32=prec == L.MIXED, device=DEV)
        b = torch.from_numpy(w["b"]).to(DEV)
        p = params(w["interval"], s, nu, 1e-10, prec)
        st1, x1, r1, nbytes = solve_with_workspace(M, b, p)
        assert nbytes <= L.STATIC_SCRATCH_BYTES
        st2, x2, r2 = solve_static(M, b, p)
        torch.cuda.synchronize()
        assert st1 == st2 == L.OK, (st1, st2, L.last_error())
        assert r1.status == r2.status == L.OK
        assert r1.outer_iters == r2.outer_iters > 0
        assert r1.refinements == r2.refinements
        assert r1.inner_iters_total == r2.inner_iters_total
        assert r1.relres == r2.relres and r1.relres_true == r2.relres_true
        assert r2.relres_true <= 2e-10
        assert torch.equal(x1, x2)
        assert r2.device_ms > 0.0
        M.close()


def test_static_solve_rejects_what_it_cannot_do():
    w = si.workload("poisson7", N=128)     # workspace of about 200 MiB
    M = P.Matrix.from_csr(w["A"], device=DEV)
    b = torch.from_numpy(w["b"]).to(DEV)
    p = params(w["interval"], 4, 2, 1e-8)
    st, x, res = solve_static(M, b, p)
    assert st == L.ERR_WORKSPACE and res.status == L.ERR_WORKSPACE
    assert "static scratch" in L.last_error()
    assert torch.count_nonzero(x).item() == 0
    M.close()
    w = si.workload("poisson5", N=16)
    M = P.Matrix.from_csr(w["A"], device=DEV)
    b = torch.from_numpy(w["b"]).to(DEV)
    for field in ("profile", "use_graph"):
        p = params(w["interval"], 4, 2, 1e-8)
        setattr(p, field, 1)
        st, x, res = solve_static(M, b, p)
        assert st == L.ERR_UNSUPPORTED, field
    # a NULL poll buffer is an argument error, as for sspcg_solve
    p = params(w["interval"], 4, 2, 1e-8)
    x = torch.zeros(M.n, dtype=torch.float64, device=DEV)
    res = L.Result()
    assert L.lib().sspcg_solve_static(M.handle, _p(b), _p(x), ctypes.byref(p), None, _stream(),
                                      ctypes.byref(res)) == L.ERR_ARG
    M.close()
