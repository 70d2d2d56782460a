"""The C ABI library: symbols, struct layouts and host-side argument checks.

None of these tests needs a GPU: every call here returns before any HIP call.
"""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_2603_09790_amd as P
from paper_2603_09790_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sspcg.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return re.findall(r"\b(sspcg_[a-z0-9_]+)\s*\(", text)


def test_every_declared_symbol_is_exported():
    decl = header_functions()
    assert decl == L.EXPORTS
    lib = ctypes.CDLL(L.LIB_PATH)
    for name in decl:
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (sspcg_\w+)", out))
    assert exported == set(decl)


def test_struct_layouts_match_header():
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "sspcg.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %d\n", sizeof(sspcg_params),
         offsetof(sspcg_params, inner_tol), offsetof(sspcg_params, check_every),
         offsetof(sspcg_params, basis), sizeof(sspcg_result),
         offsetof(sspcg_result, inner_iters_total), offsetof(sspcg_result, relres),
         offsetof(sspcg_result, relres_true), offsetof(sspcg_result, device_ms),
         sizeof(sspcg_profile), SSPCG_POLL_BYTES);
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe],
                       check=True)
        vals = list(map(int, subprocess.run([exe], capture_output=True, text=True,
                                            check=True).stdout.split()))
    assert vals == [ctypes.sizeof(L.Params), L.Params.inner_tol.offset,
                    L.Params.check_every.offset, L.Params.basis.offset, ctypes.sizeof(L.Result),
                    L.Result.inner_iters_total.offset, L.Result.relres.offset,
                    L.Result.relres_true.offset, L.Result.device_ms.offset,
                    ctypes.sizeof(L.Profile), L.POLL_BYTES]


def test_version_status_defaults():
    lib = P.lib()
    hdr = open(os.path.join(ROOT, "include", "sspcg.h")).read()
    assert lib.sspcg_abi_version() == int(re.search(r"#define SSPCG_ABI_VERSION (\d+)", hdr).group(1))
    assert L.status_string(0) == "ok"
    assert "breakdown" in L.status_string(-3)
    assert L.status_string(12345) == "unknown status"
    p = L.Params()
    lib.sspcg_default_params(ctypes.byref(p))
    assert (p.s, p.sweeps, p.tol, p.max_outer, p.check_every) == (4, 2, 1e-8, 20000, 8)


def test_matrix_memory_queries():
    """The matrix's device memory is the caller's: a closed-form scratch size
    for the analysis, then the exact aux size (argument errors are caught on
    the host, before any HIP call)."""
    lib = P.lib()
    # analysis area: a flag word, per 64-row slice its longest row, its
    # offset-union length and a union of up to 32 offsets (int32 each)
    for n in (1, 64, 65, 4096, 7077888):
        slices = (n + 63) // 64
        per = (4 * slices + 255) // 256 * 256
        assert lib.sspcg_matrix_scratch_bytes(n) == 256 + 2 * per + (128 * slices + 255) // 256 * 256
    sz = ctypes.c_size_t(123)
    A = ctypes.c_void_p(256)
    scratch = ctypes.c_void_p(4096)
    assert lib.sspcg_matrix_aux_bytes(0, 0, None, None, None, 0, scratch, 1 << 20, None,
                                      ctypes.byref(sz)) == L.ERR_ARG
    assert sz.value == 0
    assert lib.sspcg_matrix_aux_bytes(4, 4, A, A, A, 0, scratch, 1 << 20, None, None) == L.ERR_ARG
    assert lib.sspcg_matrix_aux_bytes(4, 4, A, A, A, 0, None, 1 << 20, None,
                                      ctypes.byref(sz)) == L.ERR_ARG
    assert lib.sspcg_matrix_aux_bytes(4, 4, A, A, A, 0, ctypes.c_void_p(4100), 1 << 20, None,
                                      ctypes.byref(sz)) == L.ERR_ARG
    assert lib.sspcg_matrix_aux_bytes(4, 4, A, A, A, 0, scratch, 16, None,
                                      ctypes.byref(sz)) == L.ERR_WORKSPACE
    assert lib.sspcg_matrix_aux_bytes(4, 4, A, A, A, 8, scratch, 1 << 20, None,
                                      ctypes.byref(sz)) == L.ERR_ARG
    h = ctypes.c_void_p()
    assert lib.sspcg_matrix_create(4, 4, A, A, A, 0, None, 1 << 20, None,
                                   ctypes.byref(h)) == L.ERR_ARG
    assert lib.sspcg_matrix_create(4, 4, A, A, A, 0, ctypes.c_void_p(4100), 1 << 20, None,
                                   ctypes.byref(h)) == L.ERR_ARG
    assert lib.sspcg_matrix_create(4, 4, A, A, A, 0, scratch, 16, None,
                                   ctypes.byref(h)) == L.ERR_WORKSPACE
    assert h.value is None


def test_solvers_need_a_pinned_poll_buffer():
    """The solvers poll through caller memory: NULL or misaligned is refused
    before anything is enqueued (the pinned-memory check itself needs a GPU)."""
    import torch
    lib = P.lib()
    if torch.cuda.is_available():
        pytest.skip("the handle below is fake; the GPU suite covers real solves")
    p = L.Params()
    lib.sspcg_default_params(ctypes.byref(p))
    res = L.Result()
    assert lib.sspcg_solve(None, None, None, ctypes.byref(p), None, 0, None, None,
                           ctypes.byref(res), None, None) == L.ERR_ARG


def test_host_side_argument_errors():
    lib = P.lib()
    h = ctypes.c_void_p()
    A = ctypes.c_void_p(256)
    aux = ctypes.c_void_p(4096)
    assert lib.sspcg_matrix_create(0, 0, None, None, None, 0, aux, 1 << 20, None,
                                   ctypes.byref(h)) == L.ERR_ARG
    assert "n >= 1" in L.last_error()
    assert lib.sspcg_matrix_create(10, 5, A, A, A, 0, aux, 1 << 20, None,
                                   ctypes.byref(h)) == L.ERR_ARG
    assert lib.sspcg_matrix_create(10, 10, ctypes.c_void_p(258), A, A, 0, aux, 1 << 20, None,
                                   ctypes.byref(h)) == L.ERR_ARG
    assert lib.sspcg_matrix_create(4, 4, A, A, A, 8, aux, 1 << 20, None,
                                   ctypes.byref(h)) == L.ERR_ARG
    assert lib.sspcg_matrix_create(4, 4, None, None, None, 0, aux, 1 << 20, None,
                                   None) == L.ERR_ARG
    p = L.Params()
    lib.sspcg_default_params(ctypes.byref(p))
    res = L.Result()
    poll = ctypes.c_void_p(4096)
    assert lib.sspcg_solve(None, None, None, ctypes.byref(p), None, 0, poll, None,
                           ctypes.byref(res), None, None) == L.ERR_ARG
    assert lib.sspcg_pcg_solve(None, None, None, ctypes.byref(p), None, 0, poll, None,
                               ctypes.byref(res), None) == L.ERR_ARG
    sz = ctypes.c_size_t()
    assert lib.sspcg_workspace_bytes(None, ctypes.byref(p), ctypes.byref(sz)) == L.ERR_ARG
    X = ctypes.c_void_p(256)
    st = ctypes.c_void_p(256)
    assert lib.sspcg_fgs(0, 1, X, X, 2, 0.0, 0, X, st, None) == L.ERR_ARG
    assert lib.sspcg_fgs(17, 1, X, X, 2, 0.0, 0, X, st, None) == L.ERR_ARG
    assert lib.sspcg_fgs(4, 1, X, X, 0, 0.0, 0, X, st, None) == L.ERR_ARG
    assert lib.sspcg_fgs(4, 1, X, X, 2, 0.0, 7, X, st, None) == L.ERR_ARG
    assert lib.sspcg_fgs(4, 1, None, X, 2, 0.0, 0, X, st, None) == L.ERR_ARG
    assert lib.sspcg_fgs(4, 1, X, X, 2, -1.0, 0, X, st, None) == L.ERR_ARG
    assert lib.sspcg_gram_rect(0, 4, 0, X, X, 1, X, X, 1 << 30, None) == L.ERR_ARG
    assert lib.sspcg_gram_rect(100, 4, 0, X, X, 50, X, X, 1 << 30, None) == L.ERR_ARG
    assert lib.sspcg_gram_rect(100, 4, 0, X, X, 128, X, X, 16, None) == L.ERR_WORKSPACE
    assert lib.sspcg_gram_rect(100, 4, 5, X, X, 128, X, X, 1 << 30, None) == L.ERR_ARG
    assert lib.sspcg_block_update_gram(100, 0, 0, X, X, X, X, None, X, 128, X, X, X, 1 << 30,
                                       None) == L.ERR_ARG
    assert lib.sspcg_spmv(None, 0, X, X, None) == L.ERR_ARG
    assert lib.sspcg_mpk(None, 0, X, 4, 0.0, 2.0, 0, X, X, 128, None) == L.ERR_ARG
    assert lib.sspcg_csr_value_grad(None, X, X, X, None) == L.ERR_ARG
    assert lib.sspcg_diffusion7_assemble(None, X, X, None) == L.ERR_ARG
    assert lib.sspcg_diffusion7_theta_grad(None, X, X, X, None) == L.ERR_ARG
    assert lib.sspcg_stream_triad(-1, X, X, 1.0, X, None) == L.ERR_ARG
    assert lib.sspcg_stream_triad(8, ctypes.c_void_p(264), X, 1.0, X, None) == L.ERR_ARG
    assert lib.sspcg_stream_triad(8, X, X, 1.0, None, None) == L.ERR_ARG
    assert lib.sspcg_stream_triad(0, None, None, 1.0, None, None) == L.OK
    assert lib.sspcg_matrix_destroy(None) == L.OK
    assert lib.sspcg_kernel_work_bytes(4) >= 16 * 4096 * 8


def test_package_has_no_cpu_fallback():
    """The product path never imports the oracle or the input generators."""
    pkg = os.path.join(ROOT, "paper_2603_09790_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(import|from)\s+(oracle|sspcg_inputs)\b", text, re.M), f
