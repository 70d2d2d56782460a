"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds api.hip (argument checking, workspace layout, the solve drivers) with
the sanitizers on its host code, links it with the library's other objects
and a C driver, and runs the driver on the CPU: every C-ABI entry point is
called on its host-only paths (version, status strings, default parameters,
size queries, and each argument error, which is reported before any HIP
call).  An invalid access or undefined behaviour aborts the driver.
"""
import os
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2603_09790_amd")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"

DRIVER = r'''
#include <stdio.h>
#include <string.h>
#include "sspcg.h"

static int fails = 0;
#define EXPECT(call, code) do { int rc_ = (call); \
    if (rc_ != (code)) { fprintf(stderr, "line %d: %s -> %d, expected %d\n", __LINE__, #call, rc_, (code)); ++fails; } \
    else if ((code) < 0 && strlen(sspcg_last_error()) == 0) { fprintf(stderr, "line %d: no error text\n", __LINE__); ++fails; } \
} while (0)

int main(void) {
    void* A = (void*)256;           /* never dereferenced: rejected before use */
    void* X = (void*)256;
    void* mis = (void*)258;         /* misaligned */
    sspcg_matrix* h = 0;
    sspcg_params p;
    sspcg_result res;
    size_t sz = 0;
    if (sspcg_abi_version() < 1) ++fails;
    for (int s = -7; s <= 2; ++s) if (!sspcg_status_string(s) || !sspcg_status_string(s)[0]) ++fails;
    sspcg_default_params(0);
    sspcg_default_params(&p);
    if (p.s < 1 || p.sweeps < 1 || !(p.tol > 0)) ++fails;
    for (int n = 1; n < 100000; n = n * 7 + 3) if (sspcg_matrix_scratch_bytes(n) < 256) ++fails;
    for (int s = 1; s <= 16; ++s) if (sspcg_kernel_work_bytes(s) == 0) ++fails;
    EXPECT(sspcg_matrix_aux_bytes(0, 0, 0, 0, 0, 0, X, 1 << 20, 0, &sz), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_aux_bytes(10, 5, A, A, A, 0, X, 1 << 20, 0, &sz), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_aux_bytes(10, 10, A, A, A, 0, X, 1 << 20, 0, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_create(0, 0, 0, 0, 0, 0, X, 1 << 20, 0, &h), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_create(10, 5, A, A, A, 0, X, 1 << 20, 0, &h), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_create(10, 10, mis, A, A, 0, X, 1 << 20, 0, &h), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_create(4, 4, A, A, A, 8, X, 1 << 20, 0, &h), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_create(4, 4, 0, 0, 0, 0, X, 1 << 20, 0, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_update_values(0, A, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_matrix_destroy(0), SSPCG_OK);
    EXPECT(sspcg_workspace_bytes(0, &p, &sz), SSPCG_ERR_ARG);
    EXPECT(sspcg_solve(0, 0, 0, &p, 0, 0, X, 0, &res, 0, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_solve(0, 0, 0, &p, 0, 0, X, 0, 0, 0, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_solve_static(0, 0, 0, &p, X, 0, &res), SSPCG_ERR_ARG);
    EXPECT(sspcg_pcg_solve(0, 0, 0, &p, 0, 0, X, 0, &res, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_interval_work_bytes(0, 20, &sz), SSPCG_ERR_ARG);
    EXPECT(sspcg_fgs(0, 1, X, X, 2, 0.0, 0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_fgs(17, 1, X, X, 2, 0.0, 0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_fgs(4, 1, X, X, 0, 0.0, 0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_fgs(4, 1, X, X, 2, 0.0, 7, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_fgs(4, 1, 0, X, 2, 0.0, 0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_fgs(4, 1, X, X, 2, -1.0, 0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_gram_rect(0, 4, 0, X, X, 1, X, X, 1 << 30, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_gram_rect(100, 4, 0, X, X, 50, X, X, 1 << 30, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_gram_rect(100, 4, 0, X, X, 128, X, X, 16, 0), SSPCG_ERR_WORKSPACE);
    EXPECT(sspcg_gram_rect(100, 4, 5, X, X, 128, X, X, 1 << 30, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_block_update_gram(100, 0, 0, X, X, X, X, 0, X, 128, X, X, X, 1 << 30, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_spmv(0, 0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_mpk(0, 0, X, 4, 0.0, 2.0, 0, X, X, 128, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_xr_update(0, 4, 0, X, X, X, 128, X, X, X, X, X, 1 << 30, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_csr_value_grad(0, X, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_diffusion7_assemble(0, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_diffusion7_theta_grad(0, X, X, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_stream_triad(-1, X, X, 1.0, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_stream_triad(8, mis, X, 1.0, X, 0), SSPCG_ERR_ARG);
    EXPECT(sspcg_stream_triad(0, 0, 0, 1.0, 0, 0), SSPCG_OK);
    printf("driver done, %d failures\n", fails);
    return fails ? 1 : 0;
}
'''


def _objects():
    build = os.path.join(PKG, "_build")
    names = ["sell.o", "block.o", "fgs.o", "diff.o", "interval.o", "stream.o"]
    objs = [os.path.join(build, f) for f in names]
    if not all(os.path.exists(o) for o in objs):
        pytest.skip("build the library first (python paper_2603_09790_amd/build.py)")
    return objs


def test_abi_host_code_under_asan_ubsan():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain not found")
    objs = _objects()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    with tempfile.TemporaryDirectory() as tmp:
        api_o = os.path.join(tmp, "api_san.o")
        r = subprocess.run([HIPCC, "-O1", "-g", "--offload-arch=gfx950", "-fPIC", "-std=c++17",
                            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *san,
                            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
                            "-c", os.path.join(PKG, "csrc", "api.hip"), "-o", api_o],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        drv_c = os.path.join(tmp, "driver.c")
        with open(drv_c, "w") as f:
            f.write(DRIVER)
        exe = os.path.join(tmp, "driver")
        # the host link (no device code of its own) with clang's sanitizer runtimes
        r = subprocess.run([CLANG, "-O1", "-g", "-fsanitize=address,undefined",
                            "-I", os.path.join(ROOT, "include"), drv_c, api_o, *objs,
                            "-L/opt/rocm/lib", "-lamdhip64", "-lstdc++", "-lm",
                            "-Wl,-rpath,/opt/rocm/lib", "-o", exe],
                           capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-3000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-3000:])
        assert "0 failures" in r.stdout
