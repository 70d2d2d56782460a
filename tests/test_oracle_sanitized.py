"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code).

Builds sspcg_oracle.c together with a small C driver that runs every solver
entry on a tiny 2D Poisson system (and the FGS/Cholesky breakdown paths),
then runs it; any invalid access or undefined behaviour aborts the driver.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

DRIVER = r'''
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
typedef struct { int32_t status, iters, refinements, inner_total; double relres, relres_true; } or_result;
int or_sspcg(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*,
             int, int, double, double, double, int, int, double, int, double*, or_result*);
int or_pcg(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*,
           double, int, double*, or_result*);
int or_sspcg_mixed(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*,
                   int, int, double, double, double, double, int, int, double*, or_result*);
int or_fgs(int, int, const double*, const double*, int, double*);
int or_chol_solve(int, int, const double*, const double*, double*);
void or_diffusion7_assemble(int64_t, const int32_t*, const int32_t*, const double*, double*);
void or_csr_value_grad(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*);
void or_diffusion7_theta_grad(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*);

int main(void) {
    const int N = 12, n = N * N;
    int32_t* rp = malloc(sizeof(int32_t) * (n + 1));
    int32_t* col = malloc(sizeof(int32_t) * 5 * n);
    double* val = malloc(sizeof(double) * 5 * n);
    int e = 0;
    rp[0] = 0;
    for (int y = 0; y < N; ++y) for (int x = 0; x < N; ++x) {
        const int i = x + N * y;
        if (y > 0) { col[e] = i - N; val[e++] = -1; }
        if (x > 0) { col[e] = i - 1; val[e++] = -1; }
        col[e] = i; val[e++] = 4;
        if (x < N - 1) { col[e] = i + 1; val[e++] = -1; }
        if (y < N - 1) { col[e] = i + N; val[e++] = -1; }
        rp[i + 1] = e;
    }
    double* b = malloc(sizeof(double) * n);
    double* x = calloc(n, sizeof(double));
    double* hist = malloc(sizeof(double) * 3 * 2000);
    for (int i = 0; i < n; ++i) b[i] = sin(0.1 * i);
    const double c = cos(3.14159265358979 / (N + 1));
    or_result r;
    int bad = 0;
    for (int s = 1; s <= 16; s += 5)
        for (int basis = 0; basis < 2; ++basis) {
            for (int i = 0; i < n; ++i) x[i] = 0;
            or_sspcg(n, rp, col, val, b, x, s, 3, 1 - c, 1 + c, 1e-9, 2000, 0, 1e-3, basis, hist, &r);
            if (r.status < 0) bad |= 1;
        }
    for (int i = 0; i < n; ++i) x[i] = 0;
    or_sspcg(n, rp, col, val, b, x, 4, 1, 1 - c, 1 + c, 1e-9, 2000, 1, 0.0, 0, hist, &r);
    if (r.status != 0) bad |= 2;
    for (int i = 0; i < n; ++i) x[i] = 0;
    or_pcg(n, rp, col, val, b, x, 1e-10, 1000, hist, &r);
    if (r.status != 0) bad |= 4;
    for (int i = 0; i < n; ++i) x[i] = 0;
    or_sspcg_mixed(n, rp, col, val, b, x, 4, 2, 1 - c, 1 + c, 1e-10, 1e-4, 2000, 20, hist, &r);
    if (r.status != 0) bad |= 8;
    double W[9] = {1, 0, 0, 0, 0, 0, 0, 0, 1}, m[3] = {1, 1, 1}, a[3];
    if (or_fgs(3, 1, W, m, 2, a) != -3) bad |= 16;
    if (or_chol_solve(3, 1, W, m, a) != -3) bad |= 32;
    double* theta = malloc(sizeof(double) * n);
    double* g = malloc(sizeof(double) * 5 * n);
    double* gt = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) theta[i] = 0.1 * sin(i);
    or_diffusion7_assemble(n, rp, col, theta, val);
    or_csr_value_grad(n, rp, col, b, b, g);
    or_diffusion7_theta_grad(n, rp, col, theta, g, gt);
    printf("done %d\n", bad);
    free(rp); free(col); free(val); free(b); free(x); free(hist); free(theta); free(g); free(gt);
    return bad;
}
'''


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan():
    with tempfile.TemporaryDirectory() as d:
        drv = os.path.join(d, "driver.c")
        exe = os.path.join(d, "driver")
        open(drv, "w").write(DRIVER)
        cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-ffp-contract=off", drv, os.path.join(ROOT, "oracle", "sspcg_oracle.c"),
               "-o", exe, "-lm"]
        subprocess.run(cmd, check=True, capture_output=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0")
        out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
        assert out.returncode == 0, out.stdout + out.stderr[-3000:]
        assert "done 0" in out.stdout
