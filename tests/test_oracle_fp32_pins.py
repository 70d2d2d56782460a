"""Direct pins of the oracle's FP32-storage pieces (the mixed-precision form).

The refinement's inner solve stores values, basis, directions and residual
in FP32 and forms every result in FP64 from the exactly converted operands,
rounding once on store.  These tests pin each FP32 piece on its own, not only
through the end result of the self-correcting refinement loop:

* the block update (Q <- Z + Q beta, AQ <- AZ + AQ beta) and the x/r update
  (x += Q alpha, r -= AQ alpha) of Algorithm 1: bit for bit the FP32
  rounding of the FP64 oracle's update of the upcast operands, and within one
  FP32 unit of the rounded dense definition;
* the matrix powers kernel (Algorithm 2, Sec. 2): its basis column j is the
  Chebyshev polynomial T_j(Ah) M^{-1} r with Ah = (2 M^{-1} A - (lmax + lmin)
  I) / (lmax - lmin), built densely from the FP32 values, within a first-order
  FP32 rounding bound, and each P column is A z rounded once;
* the inner solve: with s = 1 it is FP32-storage PCG and follows the FP64
  PCG iterates of the same FP32 matrix to a few FP32 units; with s = 4 it
  follows the FP64 s-step oracle on that matrix likewise.
"""
from dataclasses import replace

import numpy as np
import pytest

import oracle
import sspcg_inputs as si

U32 = 2.0 ** -24          # unit roundoff of FP32


def fp32_system(name, N):
    """The workload's matrix with its values rounded to FP32 (the FP64 copy
    holds the same numbers), FP32 1/diag and an FP32 right-hand side."""
    w = si.workload(name, N=N)
    A = w["A"]
    v32 = A.val.astype(np.float32)
    A32 = replace(A, val=v32.astype(np.float64))
    dinv32 = oracle.jacobi_inverse(A32).astype(np.float32)
    b32 = w["b"].astype(np.float32)
    return w, A, A32, v32, dinv32, b32


# ------------------------------------------------------------ block updates
@pytest.mark.parametrize("s", [1, 4, 6])
def test_fp32_block_update_is_rounded_fp64_update(s):
    rng = np.random.default_rng(30 + s)
    n = 4099
    Z, Q, AZ, AQ = (rng.normal(size=(s, n)).astype(np.float32) for _ in range(4))
    beta = rng.normal(size=(s, s))        # not symmetric: a transposed beta shows
    Q32, AQ32 = Q.copy(), AQ.copy()
    oracle.block_update(Z, Q32, AZ, AQ32, beta)
    Q64, AQ64 = Q.astype(np.float64), AQ.astype(np.float64)
    oracle.block_update(Z.astype(np.float64), Q64, AZ.astype(np.float64), AQ64, beta)
    assert np.array_equal(Q32, Q64.astype(np.float32))
    assert np.array_equal(AQ32, AQ64.astype(np.float32))
    # the definition: column j of Q' is z_j + sum_l q_l beta_lj
    for got, ref in ((Q32, Z + beta.T @ Q.astype(np.float64)),
                     (AQ32, AZ + beta.T @ AQ.astype(np.float64))):
        ref32 = ref.astype(np.float32)
        assert np.all(np.abs(got.astype(np.float64) - ref32) <= np.spacing(np.abs(ref32)))


@pytest.mark.parametrize("s", [1, 4, 6])
def test_fp32_xr_update_is_rounded_fp64_update(s):
    rng = np.random.default_rng(40 + s)
    n = 4099
    Q, AQ = (rng.normal(size=(s, n)).astype(np.float32) for _ in range(2))
    x, r = (rng.normal(size=n).astype(np.float32) for _ in range(2))
    alpha = rng.normal(size=s)
    x32, r32 = x.copy(), r.copy()
    oracle.xr_update(Q, AQ, alpha, x32, r32)
    x64, r64 = x.astype(np.float64), r.astype(np.float64)
    oracle.xr_update(Q.astype(np.float64), AQ.astype(np.float64), alpha, x64, r64)
    assert np.array_equal(x32, x64.astype(np.float32))
    assert np.array_equal(r32, r64.astype(np.float32))
    for got, ref in ((x32, x + alpha @ Q.astype(np.float64)),
                     (r32, r - alpha @ AQ.astype(np.float64))):
        ref32 = ref.astype(np.float32)
        assert np.all(np.abs(got.astype(np.float64) - ref32) <= np.spacing(np.abs(ref32)))


# ------------------------------------------------------- matrix powers kernel
@pytest.mark.parametrize("name,N,s", [("poisson5", 12, 6), ("poisson7", 8, 8),
                                      ("diffusion27", 8, 6), ("diffusion27", 8, 12)])
def test_fp32_mpk_is_chebyshev_polynomial_within_rounding(name, N, s):
    """z_j = T_j(Ah) M^{-1} r, j = 0..s-1, and p_{q+1} = A z_q.

    Bound: step q rounds p, zp and z once each (3 roundings of relative size
    <= u); an error made at step i reaches column j through the second-kind
    Chebyshev polynomial U_{j-i}(Ah) of the three-term recurrence, of size
    <= j - i + 1 on the interval, so column j carries at most
    3 u sum_{i<=j} (j-i+1) = 3 u (j+1)(j+2)/2 relative to the largest column
    so far.  P columns are FP64 sums rounded once: <= half an FP32 unit
    beyond the FP64 sum's own error.
    """
    w, A, A32, v32, dinv32, _ = fp32_system(name, N)
    lmin, lmax = w["interval"]
    r32 = np.random.default_rng(3).normal(size=A.n).astype(np.float32)
    Z, P = oracle.mpk_f32(A, v32, dinv32, r32, s, (lmin, lmax))
    M = si.to_scipy(A32).toarray()
    Ah = (2.0 * dinv32.astype(np.float64)[:, None] * M - (lmax + lmin) * np.eye(A.n)) \
        / (lmax - lmin)
    ref = [dinv32.astype(np.float64) * r32]
    ref.append(Ah @ ref[0])
    for _ in range(2, s):
        ref.append(2.0 * Ah @ ref[-1] - ref[-2])
    scale = 0.0
    for j in range(s):
        scale = max(scale, np.abs(ref[j]).max())
        bound = 3.0 * U32 * (j + 1) * (j + 2) / 2.0 * scale
        assert np.abs(Z[j] - ref[j]).max() <= bound, (j, np.abs(Z[j] - ref[j]).max() / bound)
    assert np.array_equal(P[0], r32)
    absM = np.abs(M)
    for q in range(s):
        y = M @ Z[q].astype(np.float64)
        err = np.abs(P[q + 1].astype(np.float64) - y)
        lim = 0.5 * np.spacing(np.abs(P[q + 1])) + 1e-14 * (absM @ np.abs(Z[q].astype(np.float64)))
        assert np.all(err <= lim), q


# ------------------------------------------------------------- inner solve
@pytest.mark.parametrize("name,N", [("poisson5", 12), ("diffusion27", 8)])
def test_fp32_inner_solve_s1_is_pcg(name, N):
    """s = 1: each outer iteration is one PCG step (1x1 Gram solves are exact).
    After k steps the FP32-storage iterate is the FP64 PCG iterate on the same
    FP32 matrix up to a few FP32 units (measured <= 2.3 u at k = 12)."""
    w, A, A32, v32, dinv32, b32 = fp32_system(name, N)
    for k in (1, 2, 3, 5, 8, 12):
        d, st, it = oracle.inner_sspcg_f32(A, v32, dinv32, b32, s=1, sweeps=2,
                                           interval=w["interval"], inner_tol=1e-30,
                                           max_inner=k)
        x, res = oracle.pcg(A32, b32.astype(np.float64), tol=1e-30, max_iter=k)
        assert st == oracle.NOT_CONVERGED and it == k and res["iters"] == k
        assert np.linalg.norm(d - x) <= 20 * U32 * np.linalg.norm(x), k


@pytest.mark.parametrize("name,N", [("poisson5", 12), ("diffusion27", 8)])
def test_fp32_inner_solve_follows_fp64_sspcg(name, N):
    """s = 4, nu = 2: the FP32-storage iterates follow the FP64 s-step oracle
    on the same FP32 matrix to a few FP32 units (measured <= 4 u, k <= 12),
    and the inner stop test ends at the first iterate below inner_tol."""
    w, A, A32, v32, dinv32, b32 = fp32_system(name, N)
    for k in (1, 2, 3, 5, 8, 12):
        d, st, it = oracle.inner_sspcg_f32(A, v32, dinv32, b32, s=4, sweeps=2,
                                           interval=w["interval"], inner_tol=1e-30,
                                           max_inner=k)
        x, res = oracle.sspcg(A32, b32.astype(np.float64), s=4, sweeps=2,
                              interval=w["interval"], tol=1e-30, max_outer=k)
        assert st == oracle.NOT_CONVERGED and it == k and res["iters"] == k
        assert np.linalg.norm(d - x) <= 20 * U32 * np.linalg.norm(x), k
    d, st, it = oracle.inner_sspcg_f32(A, v32, dinv32, b32, s=4, sweeps=2,
                                       interval=w["interval"], inner_tol=1e-3, max_inner=500)
    assert st == oracle.OK
    M = si.to_scipy(A32)
    rel = lambda v: np.linalg.norm(b32 - M @ v.astype(np.float64)) / np.linalg.norm(b32)
    assert rel(d) <= 1.5e-3
    dp, _, _ = oracle.inner_sspcg_f32(A, v32, dinv32, b32, s=4, sweeps=2,
                                      interval=w["interval"], inner_tol=1e-30, max_inner=it - 1)
    assert rel(dp) > 0.5e-3
