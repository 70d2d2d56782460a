"""Guard bytes around every caller buffer the library writes.

The workspace of a solve, the matrix layout buffer (aux) and the kernel-level
work buffer are handed over at their exact query sizes inside larger
allocations filled with a byte pattern; after matrix creation, FP64, mixed
and PCG solves and the kernel-level calls, every byte outside the handed-over
range must still hold the pattern (a kernel that wrote past its buffer would
change them).
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
PAD = 1 << 16
FILL = 0xA5


def guarded(nbytes):
    """(buffer, pointer at PAD into it, exact size): PAD guard bytes each side."""
    buf = torch.full((PAD + nbytes + PAD,), FILL, dtype=torch.uint8, device=DEV)
    return buf, ctypes.c_void_p(buf.data_ptr() + PAD), nbytes


def guards_intact(buf, nbytes):
    torch.cuda.synchronize()
    head, tail = buf[:PAD], buf[PAD + nbytes:]
    return bool(torch.all(head == FILL).item()) and bool(torch.all(tail == FILL).item())


def _p(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@pytest.mark.parametrize("kind,N", [("27pt", 20), ("7pt", 21), ("5pt", 45)])
def test_buffers_are_not_overrun(kind, N):
    lib = L.lib()
    kap = np.exp(si.theta_field(N ** (2 if kind == "5pt" else 3)))
    A = si.stencil(kind, N, kap)
    b = torch.from_numpy(si.rhs_normal(A.n)).to(DEV)
    rp = torch.from_numpy(A.row_ptr).to(DEV)
    col = torch.from_numpy(A.col).to(DEV)
    val = torch.from_numpy(A.val).to(DEV)
    args = (A.n, A.nnz, _p(rp), _p(col), _p(val), L.MATRIX_FP32)
    scratch = torch.empty(lib.sspcg_matrix_scratch_bytes(A.n), dtype=torch.uint8, device=DEV)
    need = ctypes.c_size_t()
    assert lib.sspcg_matrix_aux_bytes(*args, _p(scratch), scratch.numel(), _stream(),
                                      ctypes.byref(need)) == L.OK
    abuf, aptr, an = guarded(need.value)
    h = ctypes.c_void_p()
    assert lib.sspcg_matrix_create(*args, aptr, an, _stream(), ctypes.byref(h)) == L.OK
    assert guards_intact(abuf, an)
    interval = si.lanczos_bounds(A)
    poll = torch.empty(L.POLL_BYTES, dtype=torch.uint8, pin_memory=True)
    for precision, s in ((L.FP64, 6), (L.MIXED, 4), (L.FP64, 16)):
        p = L.Params()
        lib.sspcg_default_params(ctypes.byref(p))
        p.s, p.sweeps, p.tol, p.precision = s, 2, 1e-10, precision
        p.lambda_min, p.lambda_max = interval
        wb = ctypes.c_size_t()
        assert lib.sspcg_workspace_bytes(h, ctypes.byref(p), ctypes.byref(wb)) == L.OK
        wbuf, wptr, wn = guarded(wb.value)
        x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
        res = L.Result()
        hist = (ctypes.c_double * (L.HIST_STRIDE * p.max_outer))()
        st = lib.sspcg_solve(h, _p(b), _p(x), ctypes.byref(p), wptr, wn, _p(poll), _stream(),
                             ctypes.byref(res), hist, None)
        assert st in (L.OK, L.NOT_CONVERGED), L.last_error()
        assert guards_intact(wbuf, wn), (precision, s)
        assert guards_intact(abuf, an)
    # classical PCG
    p = L.Params()
    lib.sspcg_default_params(ctypes.byref(p))
    wb = ctypes.c_size_t()
    assert lib.sspcg_workspace_bytes(h, ctypes.byref(p), ctypes.byref(wb)) == L.OK
    wbuf, wptr, wn = guarded(wb.value)
    x = torch.zeros(A.n, dtype=torch.float64, device=DEV)
    res = L.Result()
    assert lib.sspcg_pcg_solve(h, _p(b), _p(x), ctypes.byref(p), wptr, wn, _p(poll), _stream(),
                               ctypes.byref(res), None) == L.OK
    assert guards_intact(wbuf, wn)
    # kernel-level reductions with their exact work buffer
    s = 6
    ld = P.leading_dim(A.n)
    kbuf, kptr, kn = guarded(lib.sspcg_kernel_work_bytes(s))
    Q = torch.randn((s, ld), dtype=torch.float64, device=DEV)
    AZ = torch.randn_like(Q)
    B2 = torch.empty((s, s), dtype=torch.float64, device=DEV)
    assert lib.sspcg_gram_rect(A.n, s, L.F64, _p(Q), _p(AZ), ld, _p(B2), kptr, kn,
                               _stream()) == L.OK
    assert guards_intact(kbuf, kn)
    assert lib.sspcg_matrix_destroy(h) == L.OK
    assert guards_intact(abuf, an)
