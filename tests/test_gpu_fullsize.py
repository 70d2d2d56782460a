"""Parity at the benchmark's full size: 27-point diffusion on 192^3.

n = 7,077,888, nnz = 189,119,224, the launch configuration the benchmark
times.  The oracle recomputes what the host can afford: SpMV rows sampled at
random, one matrix powers kernel, the Gram reductions of that block and the
first two outer iterations of the FP64 solve; the complete FP64 and mixed
solves are checked by their true residual.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_09790_amd as P
import sspcg_inputs as si

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
N = 192


@pytest.fixture(scope="module")
def big():
    A = si.stencil("27pt", N, si.coeff_blocks(N))
    b = si.rhs_normal(A.n)
    interval = si.lanczos_bounds(A)
    M = P.Matrix.from_csr(A, fp32=True, device=DEV)
    return A, b, interval, M


def sampled_rows(A, x, rows):
    out = np.empty(len(rows))
    scale = np.empty(len(rows))
    for t, i in enumerate(rows):
        a, e = A.row_ptr[i], A.row_ptr[i + 1]
        v, c = A.val[a:e], A.col[a:e]
        acc = 0.0
        for k in range(e - a):
            acc += v[k] * x[c[k]]
        out[t] = acc
        scale[t] = np.abs(v) @ np.abs(x[c])
    return out, scale


def test_layout_of_full_workload(big):
    A, _, _, M = big
    info = M.info()
    assert A.nnz == (3 * N - 2) ** 3
    assert info["slices"] == info["shared_slices"] == A.n // 64
    # symmetric half storage: the diagonal and the 13 upper offsets per row
    assert info["symmetric"] == 1 and info["slots"] == 14 * A.n
    assert info["slots"] <= 1.02 * (A.nnz + A.n) / 2


def test_spmv_sampled_rows(big):
    A, _, _, M = big
    rng = np.random.default_rng(30)
    x = rng.normal(size=A.n)
    y = P.spmv(M, torch.from_numpy(x).to(DEV)).cpu().numpy()
    rows = np.concatenate([rng.integers(0, A.n, 3000), [0, 1, N - 1, N * N, A.n - 1]])
    ref, scale = sampled_rows(A, x, rows)
    assert np.all(np.abs(y[rows] - ref) <= 1e-14 * scale)
    x32 = x.astype(np.float32)
    y32 = P.spmv(M, torch.from_numpy(x32).to(DEV)).cpu().numpy()
    ref32 = oracle.spmv_f32(A, A.val.astype(np.float32), x32)
    assert np.array_equal(y32, ref32)


def test_mpk_and_gram_full(big):
    A, b, interval, M = big
    s = 6
    dinv = oracle.jacobi_inverse(A)
    Zo, Po = oracle.mpk(A, dinv, b, s, interval)
    ld = P.leading_dim(A.n)
    Z, Pm = P.mpk(M, torch.from_numpy(b).to(DEV), s, interval, ld=ld)
    Zh, Ph = Z.cpu().numpy()[:, :A.n], Pm.cpu().numpy()[:, :A.n]
    for j in range(s):
        assert np.abs(Zh[j] - Zo[j]).max() <= 1e-12 * np.abs(Zo[j]).max()
        assert np.abs(Ph[j + 1] - Po[j + 1]).max() <= 1e-12 * np.abs(Po[j + 1]).max()
    Q = torch.empty_like(Z)
    AQ = torch.empty_like(Z)
    W, b1 = P.block_update_gram(A.n, Z, Q, Pm[1:], AQ, None, Pm[0])
    Wo, b1o = oracle.gram(Zh, Ph[1:], Ph[0])
    scale = np.abs(Zh) @ np.abs(Ph[1:]).T
    assert np.all(np.abs(W.cpu().numpy() - Wo) <= 1e-12 * scale)
    scale_b = np.abs(Zh) @ np.abs(Ph[0])
    assert np.all(np.abs(b1.cpu().numpy() - b1o) <= 1e-12 * scale_b)


def test_first_outer_iterations_full(big):
    A, b, interval, M = big
    x, info = P.solve(M, torch.from_numpy(b).to(DEV), s=6, sweeps=2, interval=interval,
                      tol=1e-30, max_outer=2)
    xo, ro = oracle.sspcg(A, b, s=6, sweeps=2, interval=interval, tol=1e-30, max_outer=2)
    assert info["outer_iters"] == ro["iters"] == 2
    xh = x.cpu().numpy()
    assert np.linalg.norm(xh - xo) <= 1e-10 * np.linalg.norm(xo)
    assert abs(info["relres"] - ro["relres"]) <= 1e-10 * ro["relres"]


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_full_solve_true_residual(big, precision):
    A, b, interval, M = big
    x, info = P.solve(M, torch.from_numpy(b).to(DEV), s=6, sweeps=2, interval=interval,
                      tol=1e-8, precision=precision)
    assert info["status"] == P.OK
    r = b - oracle.spmv(A, x.cpu().numpy())
    rel = np.linalg.norm(r) / np.linalg.norm(b)
    # the recursive residual may drift from the true one by rounding
    assert rel <= 1.5e-8
    print(f"{precision}: {info['outer_iters']} iterations, {info['device_ms']:.1f} ms, "
          f"true relative residual {rel:.3e}")


def test_device_interval_full(big):
    """Device Lanczos and power estimates at full size against the oracle's."""
    A, _, interval, M = big
    v0 = si.start_vector(A.n)
    out = P.interval(M, torch.from_numpy(v0).to(DEV), method="lanczos", steps=20)
    lo, hi, k = oracle.lanczos_bounds(A, v0, 20)
    assert out["steps"] == k == 20
    assert abs(out["interval"][0] - lo) <= 1e-9 * lo and abs(out["interval"][1] - hi) <= 1e-9 * hi
    # the fixture's interval is the same estimate from the input generator
    assert abs(interval[0] - lo) <= 1e-9 * lo and abs(interval[1] - hi) <= 1e-9 * hi
    pw = P.interval(M, torch.from_numpy(v0).to(DEV), method="power", steps=50, rtol=1e-3)
    _, phi, pk, _ = oracle.power_bounds(A, v0, rtol=1e-3, max_iter=50)
    assert abs(pw["interval"][1] - phi) <= 1e-12 * phi and pw["steps"] == pk
