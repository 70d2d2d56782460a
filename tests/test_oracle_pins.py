"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test checks the oracle against the mathematics or a library routine:
dense direct solves, exact termination on operators with few eigenvalues,
the paper's closed forms (moment representation of the Chebyshev Gram
matrix, FGS residual formula and rate, Ruhe's FGS/MGS equivalence, the
Gram/basis condition-number identity) and derived invariants (A-norm error
decrease, conjugacy defect).  A dropped term, wrong sign or transposed
operand in the oracle's MPK, Gram, FGS or updates fails at least one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse.linalg as spl
from numpy.polynomial import chebyshev as npcheb

import oracle
import sspcg_inputs as si
from sspcg_inputs import CSR
from oracle_trace import trace


def dense_csr(M: np.ndarray) -> CSR:
    """Full-pattern CSR of a dense matrix (every entry stored)."""
    n = M.shape[0]
    rp = np.arange(0, n * n + 1, n, dtype=np.int32)
    col = np.tile(np.arange(n, dtype=np.int32), n)
    return CSR(n, rp, col, np.ascontiguousarray(M.reshape(-1), dtype=np.float64), (1, 1, n))


def sym_scaled(A: CSR):
    """Dense D^{-1/2} A D^{-1/2}, its eigen-decomposition and D^{-1/2}."""
    M = si.to_scipy(A).toarray()
    dh = 1.0 / np.sqrt(np.diag(M))
    B = M * np.outer(dh, dh)
    lam, V = np.linalg.eigh(B)
    return M, B, lam, V, dh


def few_eigenvalue_spd(n_blocks=(5, 4, 3), eps=(0.15, 0.1, 0.2), seed=11):
    """SPD matrix whose Jacobi-scaled form has exactly 2 eigenvalues per block.

    B = blockdiag(I + e (J - I)) has unit diagonal and eigenvalues 1 + e(m-1)
    and 1 - e per block; A = S B S with a random positive diagonal S has
    diag(A) = S^2, so D^{-1/2} A D^{-1/2} = B.
    """
    blocks = [np.eye(m) + e * (np.ones((m, m)) - np.eye(m)) for m, e in zip(n_blocks, eps)]
    B = sla.block_diag(*blocks)
    S = np.diag(np.random.default_rng(seed).uniform(0.5, 3.0, B.shape[0]))
    distinct = sorted({round(1 + e * (m - 1), 12) for m, e in zip(n_blocks, eps)}
                      | {round(1 - e, 12) for e in eps})
    return S @ B @ S, len(distinct)


# ---------------------------------------------------------------- SpMV, Jacobi
def test_spmv_matches_scipy():
    A = si.stencil("27pt", 9, si.coeff_blocks(9, block=3))
    x = np.random.default_rng(0).normal(size=A.n)
    y = oracle.spmv(A, x)
    ref = si.to_scipy(A) @ x
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()


def test_spmv_f32_is_rounded_exact_sum():
    A = si.stencil("7pt", 10, np.exp(si.theta_field(1000)))
    v32 = A.val.astype(np.float32)
    x32 = np.random.default_rng(1).normal(size=A.n).astype(np.float32)
    y = oracle.spmv_f32(A, v32, x32)
    # exact products of FP32 numbers in FP64, summed by scipy, rounded once
    S = si.to_scipy(CSR(A.n, A.row_ptr, A.col, v32.astype(np.float64), A.shape3))
    ref = (S @ x32.astype(np.float64)).astype(np.float32)
    ulp = np.spacing(np.abs(ref))
    assert np.all(np.abs(y.astype(np.float64) - ref) <= ulp)
    assert np.mean(y == ref) > 0.999


def test_diagonal_rejects_nonpositive():
    A = si.poisson5(5)
    bad = CSR(A.n, A.row_ptr, A.col, A.val.copy(), A.shape3)
    bad.val[0] = -bad.val[0]
    with pytest.raises(ValueError):
        oracle.jacobi_inverse(bad)


# ------------------------------------------------ Chebyshev Gram moment form
@pytest.mark.parametrize("s", [2, 4, 6, 8])
def test_first_gram_matches_moment_representation(s):
    """W = Z^T A Z of the raw Chebyshev block equals (mu_{i+j-2} + mu_|i-j|)/2.

    Left-preconditioned case through B = D^{-1/2} A D^{-1/2}: with
    c = V^T D^{-1/2} r and the scaled eigenvalues lh = (2l - lmax - lmin)/(lmax - lmin),
    mu_p = sum_l l c_l^2 T_p(lh_l)  (Thm. gram-structure, Cor. diagonal,
    Remark on the preconditioned case).
    """
    N = 5
    A = si.stencil("7pt", N, np.exp(si.theta_field(N**3)))
    M, B, lam, V, dh = sym_scaled(A)
    lmin, lmax = lam[0] * 0.9, lam[-1] * 1.02
    r = np.random.default_rng(3).uniform(-1, 1, A.n)
    dinv = oracle.jacobi_inverse(A)
    Z, P = oracle.mpk(A, dinv, r, s, (lmin, lmax))
    W, b1 = oracle.gram(Z, P[1:], P[0])

    c = V.T @ (dh * r)
    lh = (2 * lam - lmax - lmin) / (lmax - lmin)
    mu = np.array([np.sum(lam * c**2 * npcheb.chebval(lh, [0] * p + [1])) for p in range(2 * s)])
    Wm = np.array([[0.5 * (mu[i + j] + mu[abs(i - j)]) for j in range(s)] for i in range(s)])
    assert np.abs(W - Wm).max() <= 1e-12 * np.abs(Wm).max()
    # diagonal: (mu_0 + mu_{2i-2})/2, mu_0 = z_1^T A z_1
    assert abs(mu[0] - Z[0] @ (M @ Z[0])) <= 1e-12 * abs(mu[0])
    # normalized Gram entries are bounded by one
    d = np.sqrt(np.diag(W))
    assert np.all(np.abs(W / np.outer(d, d)) <= 1 + 1e-12)
    # b1 = Z^T r
    assert np.abs(b1 - Z @ r).max() <= 1e-12 * np.abs(b1).max()
    # P columns: P_1 = r, P_{q+1} = A z_q
    assert np.array_equal(P[0], r)
    for q in range(s):
        assert np.abs(P[q + 1] - M @ Z[q]).max() <= 1e-13 * np.abs(P[q + 1]).max()


def test_mpk_basis_is_chebyshev_polynomial_of_operator():
    """z_j = T_{j-1}(Ah) M^{-1} r with Ah = alpha M^{-1}A - sigma I."""
    A = si.stencil("5pt", 6, np.exp(si.theta_field(36)))
    M = si.to_scipy(A).toarray()
    dinv = 1.0 / np.diag(M)
    lmin, lmax = 0.05, 1.9
    s = 6
    r = np.random.default_rng(4).normal(size=A.n)
    Z, _ = oracle.mpk(A, dinv, r, s, (lmin, lmax))
    Ah = (2 * (dinv[:, None] * M) - (lmax + lmin) * np.eye(A.n)) / (lmax - lmin)
    T_prev, T = np.eye(A.n), Ah.copy()
    ref = [dinv * r, Ah @ (dinv * r)]
    for _ in range(2, s):
        T_prev, T = T, 2 * Ah @ T - T_prev
        ref.append(T @ (dinv * r))
    for j in range(s):
        assert np.abs(Z[j] - ref[j]).max() <= 1e-12 * np.abs(ref[j]).max()


# ------------------------------------------------------------------- FGS
def random_spd(s, seed, cond=50.0):
    rng = np.random.default_rng(seed)
    U, _ = np.linalg.qr(rng.normal(size=(s, s)))
    ev = np.geomspace(1.0, cond, s)
    D = np.diag(rng.uniform(0.2, 5.0, s))
    return D @ (U * ev) @ U.T @ D


@pytest.mark.parametrize("s", [1, 3, 6, 10, 16])
def test_fgs_residual_closed_form(s):
    """Prop. fgs-residual: rho^(nu) = (-1)^nu (L^T (I+L)^{-1})^nu m~."""
    W = random_spd(s, seed=s)
    m = np.random.default_rng(100 + s).normal(size=s)
    Dh = np.sqrt(np.diag(W))
    Wc = W / np.outer(Dh, Dh)
    L = np.tril(Wc, -1)
    mt = m / Dh
    G = L.T @ np.linalg.inv(np.eye(s) + L)
    for nu in range(1, 7):
        a, st = oracle.fgs(W, m, nu)
        assert st == oracle.OK
        rho = mt - Wc @ (Dh * a)
        ref = (-1) ** nu * np.linalg.matrix_power(G, nu) @ mt
        assert np.abs(rho - ref).max() <= 1e-13 * max(1.0, np.abs(mt).max())


def test_fgs_rate_and_limit():
    """Cor. spectral_radius: ||rho^(nu)||^(1/nu) -> rho(H); many sweeps solve W a = m."""
    s = 8
    W = random_spd(s, seed=5, cond=20.0)
    m = np.random.default_rng(6).normal(size=s)
    Dh = np.sqrt(np.diag(W))
    Wc = W / np.outer(Dh, Dh)
    L = np.tril(Wc, -1)
    H = -L.T @ np.linalg.inv(np.eye(s) + L)
    rhoH = np.max(np.abs(np.linalg.eigvals(H)))
    assert rhoH < 1.0
    # stay well above the rounding floor: rho(H)^nu >> 1e-16
    nu, dnu = 20, 20
    a, _ = oracle.fgs(W, m, nu)
    res = np.linalg.norm(m / Dh - Wc @ (Dh * a))
    a2, _ = oracle.fgs(W, m, nu + dnu)
    res2 = np.linalg.norm(m / Dh - Wc @ (Dh * a2))
    assert res2 > 1e-12
    rate = (res2 / res) ** (1 / dnu)
    assert abs(rate - rhoH) < 2e-2
    a_inf, _ = oracle.fgs(W, m, 3000)
    ref = np.linalg.solve(W, m)
    assert np.abs(a_inf - ref).max() <= 1e-10 * np.abs(ref).max()


def test_fgs_multiple_rhs_columns_independent_and_cholesky():
    s = 6
    W = random_spd(s, seed=9)
    B = np.random.default_rng(10).normal(size=(s, s))
    X, st = oracle.fgs(W, B, 3)
    for c in range(s):
        xc, _ = oracle.fgs(W, B[:, c], 3)
        assert np.array_equal(X[:, c], xc)
    Xc, st = oracle.chol_solve(W, B)
    assert st == oracle.OK
    assert np.abs(Xc - np.linalg.solve(W, B)).max() <= 1e-12 * np.abs(Xc).max()
    assert oracle.gram_relres(W, B, Xc) < 1e-13


def test_fgs_breakdown_and_nonfinite():
    W = np.eye(3)
    W[1, 1] = 0.0
    _, st = oracle.fgs(W, np.ones(3), 2)
    assert st == oracle.BREAKDOWN
    W = np.eye(3)
    _, st = oracle.fgs(W, np.array([1.0, np.nan, 0.0]), 2)
    assert st == oracle.NONFINITE
    Wn = np.eye(3)
    Wn[2, 0] = Wn[0, 2] = np.inf
    _, st = oracle.fgs(Wn, np.ones(3), 2)
    assert st == oracle.NONFINITE
    _, st = oracle.chol_solve(-np.eye(2), np.ones(2))
    assert st == oracle.BREAKDOWN


# ------------------------------------------------------------ Ruhe / MGS
@pytest.mark.parametrize("inner", ["standard", "A"])
def test_ruhe_one_sweep_is_mgs(inner):
    """Thm. ruhe: one FGS sweep on W a = e1 gives P a = v^(s) (MGS sweep)."""
    n, s = 40, 6
    rng = np.random.default_rng(12)
    P = rng.normal(size=(n, s)) + 0.5 * rng.normal(size=(n, 1))
    if inner == "standard":
        G = np.eye(n)
    else:
        A = si.to_scipy(si.stencil("5pt", 7, np.exp(si.theta_field(49)))).toarray()[:n, :n]
        G = A
    P = P / np.sqrt(np.einsum("ij,ij->j", P, G @ P))
    W = P.T @ G @ P
    e1 = np.zeros(s)
    e1[0] = 1.0
    a, st = oracle.fgs(W, e1, 1)
    v = P[:, 0].copy()
    for j in range(1, s):
        h = P[:, j] @ (G @ v)
        v = v - h * P[:, j]
    assert np.abs(P @ a - v).max() <= 1e-13 * np.abs(v).max()


# ------------------------------------------------------- solver-level pins
def test_sspcg_cholesky_matches_dense_solve():
    A = si.stencil("7pt", 6, np.exp(si.theta_field(216)))
    b = si.rhs_uniform(A.n)
    M = si.to_scipy(A).toarray()
    xs = np.linalg.solve(M, b)
    kappa = np.linalg.cond(M)
    lo, hi = si.lanczos_bounds(A)
    tol = 1e-13
    x, res = oracle.sspcg(A, b, s=4, sweeps=2, interval=(lo, hi), tol=tol, gram="cholesky")
    assert res["status"] == oracle.OK
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) <= 10 * kappa * tol
    x2, res2 = oracle.sspcg(A, b, s=4, sweeps=200, interval=(lo, hi), tol=tol)
    assert res2["status"] == oracle.OK
    assert np.linalg.norm(x2 - xs) / np.linalg.norm(xs) <= 10 * kappa * tol
    x3, res3 = oracle.pcg(A, b, tol=tol)
    assert res3["status"] == oracle.OK
    assert np.linalg.norm(x3 - xs) / np.linalg.norm(xs) <= 10 * kappa * tol


def test_exact_termination_few_eigenvalues():
    """Krylov methods end after as many steps as the operator has distinct
    eigenvalues; with s at least that many, one outer iteration of s-step PCG
    with an exact Gram solve gives the solution."""
    M, m = few_eigenvalue_spd()
    A = dense_csr(M)
    b = np.random.default_rng(13).normal(size=A.n)
    xs = np.linalg.solve(M, b)
    _, res = oracle.pcg(A, b, tol=1e-12)
    assert res["status"] == oracle.OK and res["iters"] <= m
    d = np.sqrt(np.diag(M))
    ev = np.linalg.eigvalsh(M / np.outer(d, d))
    x, res = oracle.sspcg(A, b, s=m, sweeps=1, interval=(ev[0] * 0.99, ev[-1] * 1.01),
                          tol=1e-12, gram="cholesky")
    assert res["status"] == oracle.OK and res["iters"] == 1
    assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs)


@pytest.mark.parametrize("sweeps", [1, 2, 5])
def test_s1_equals_pcg(sweeps):
    """s = 1: the 1x1 FGS solve is exact, so PCG-S is PCG for any sweep count."""
    w = si.workload("poisson5", N=24)
    A, b = w["A"], w["b"]
    _, r1, h1 = oracle.pcg(A, b, tol=1e-10, history=True)
    _, r2, h2 = oracle.sspcg(A, b, s=1, sweeps=sweeps, interval=w["interval"], tol=1e-10,
                             history=True)
    assert r1["iters"] == r2["iters"]
    assert np.abs(np.log(h1) - np.log(h2[:, 0])).max() < 1e-8


@pytest.mark.parametrize("s", [2, 4])
def test_exact_gram_aligns_with_pcg_every_s_steps(s):
    """With an exact Gram solve, outer iteration k of PCG-S spans the same
    Krylov space as (k+1) s PCG steps: residuals agree (Sec. 3.4 alignment)."""
    A = si.stencil("7pt", 8, np.exp(si.theta_field(512)))
    b = si.rhs_uniform(A.n)
    lo, hi = si.lanczos_bounds(A)
    _, _, hp = oracle.pcg(A, b, tol=1e-12, history=True)
    _, _, hs = oracle.sspcg(A, b, s=s, sweeps=1, interval=(lo, hi), tol=1e-12,
                            gram="cholesky", history=True)
    for k in range(3):
        assert abs(hs[k, 0] - hp[(k + 1) * s - 1]) <= 1e-10 * hp[(k + 1) * s - 1]


def test_trace_equals_oracle_loop():
    w = si.workload("poisson5", N=20)
    x, res = oracle.sspcg(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-8)
    xt, st, states = trace(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-8,
                           max_outer=10000)
    assert st == res["status"] and len(states) == res["iters"]
    assert np.array_equal(x, xt)


@pytest.mark.parametrize("sweeps", [1, 2, 30])
def test_anorm_error_never_increases(sweeps):
    """FGS from zero is exact coordinate descent on a^T W a / 2 - m^T a, so the
    A-norm error cannot grow in any outer iteration, for any sweep count."""
    A = si.stencil("7pt", 7, np.exp(si.theta_field(343)))
    b = si.rhs_uniform(A.n)
    M = si.to_scipy(A).toarray()
    xs = np.linalg.solve(M, b)
    lo, hi = si.lanczos_bounds(A)
    _, _, states = trace(A, b, s=4, sweeps=sweeps, interval=(lo, hi), tol=1e-10, max_outer=60)
    err = [math.sqrt((st["x"] - xs) @ M @ (st["x"] - xs)) for st in states]
    e0 = err[0]
    for a, c in zip(err, err[1:]):
        assert c <= a + 1e-12 * e0


def test_conjugacy_defect_and_condition_identity():
    """Q_{k+1}^T A Q_k = -(B2 - W beta)^T, and kappa(A^{1/2} Q)^2 = kappa(W).
    The oracle's history reports ||Q_{k+1}^T A Q_k||_F as its fourth column."""
    A = si.stencil("7pt", 6, np.exp(si.theta_field(216)))
    b = si.rhs_uniform(A.n)
    M = si.to_scipy(A).toarray()
    lo, hi = si.lanczos_bounds(A)
    _, _, states = trace(A, b, s=4, sweeps=2, interval=(lo, hi), tol=1e-12, max_outer=6)
    _, _, hist = oracle.sspcg(A, b, s=4, sweeps=2, interval=(lo, hi), tol=1e-12, max_outer=6,
                              history=True)
    assert hist.shape == (6, 4)
    for k in range(5):
        defect = np.linalg.norm(states[k + 1]["Q"] @ M @ states[k]["Q"].T)
        assert abs(hist[k, 3] - defect) <= 1e-9 * defect
        assert abs(hist[k, 2] * np.linalg.norm(states[k]["B2"]) - defect) <= 1e-9 * defect
    lam, V = np.linalg.eigh(M)
    Mh = (V * np.sqrt(lam)) @ V.T
    for k in range(4):
        st, nx = states[k], states[k + 1]
        lhs = nx["Q"] @ M @ st["Q"].T
        rhs = -(st["B2"] - st["W"] @ st["beta"]).T
        assert np.abs(lhs - rhs).max() <= 1e-9 * np.abs(st["B2"]).max()
        F = Mh @ st["Q"].T
        sv = np.linalg.svd(F, compute_uv=False)
        assert abs((sv[0] / sv[-1]) ** 2 / np.linalg.cond(st["W"]) - 1) < 1e-8


# ------------------------------------------------------- mixed precision
def test_mixed_pieces_are_exact_upcasts():
    """FP32-storage Gram entries equal the FP64 Gram of the upcast vectors."""
    rng = np.random.default_rng(20)
    Q = rng.normal(size=(5, 3000)).astype(np.float32)
    AQ = rng.normal(size=(5, 3000)).astype(np.float32)
    r = rng.normal(size=3000).astype(np.float32)
    W32, b32 = oracle.gram(Q, AQ, r)
    W64, b64 = oracle.gram(Q.astype(np.float64), AQ.astype(np.float64), r.astype(np.float64))
    assert np.array_equal(W32, W64) and np.array_equal(b32, b64)
    assert np.array_equal(oracle.gram_rect(Q, AQ),
                          oracle.gram_rect(Q.astype(np.float64), AQ.astype(np.float64)))


def test_mixed_refinement_reaches_fp64_accuracy():
    w = si.workload("poisson7", N=16)
    A, b = w["A"], w["b"]
    x, res = oracle.sspcg_mixed(A, b, s=4, sweeps=2, interval=w["interval"], tol=1e-10)
    assert res["status"] == oracle.OK and res["relres_true"] <= 1e-10
    assert 1 <= res["refinements"] <= 6
    r = b - si.to_scipy(A) @ x
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(b)
    xs = spl.spsolve(si.to_scipy(A).tocsc(), b)
    assert np.linalg.norm(x - xs) / np.linalg.norm(xs) < 1e-8


# ------------------------------------------------------- differentiable form
def test_diffusion7_assembly_matches_input_generator():
    N = 6
    theta = si.theta_field(N**3)
    A = si.stencil("7pt", N, np.exp(theta))
    val = oracle.diffusion7_assemble(A, theta)
    assert np.abs(val - A.val).max() <= 4e-16 * np.abs(A.val).max()
    val0 = oracle.diffusion7_assemble(A, np.zeros(A.n))
    assert np.array_equal(val0, si.poisson7(N).val)


def _loss_and_grad_dense(N, theta, b, xt):
    """Independent reference: torch autograd through a dense assembly and solve."""
    import torch
    th = torch.tensor(theta, dtype=torch.float64, requires_grad=True)
    k = torch.exp(th)
    n = N**3
    Mx = torch.zeros((n, n), dtype=torch.float64)
    idx = np.arange(n)
    z, y, x = idx // (N * N), (idx // N) % N, idx % N
    rows, cols = [], []
    for dz, dy, dx in [(0, 0, 1), (0, 1, 0), (1, 0, 0)]:
        ok = (x + dx < N) & (y + dy < N) & (z + dz < N)
        i = idx[ok]
        j = i + dx + N * dy + N * N * dz
        rows.append(i)
        cols.append(j)
    i = torch.tensor(np.concatenate(rows))
    j = torch.tensor(np.concatenate(cols))
    w = 2 * k[i] * k[j] / (k[i] + k[j])
    deg = torch.zeros(n, dtype=torch.float64).index_add(0, i, torch.ones_like(w)) \
        .index_add(0, j, torch.ones_like(w))
    Mx = Mx.index_put((i, j), -w, accumulate=True).index_put((j, i), -w, accumulate=True)
    diag = torch.zeros(n, dtype=torch.float64).index_add(0, i, w).index_add(0, j, w) \
        + (6 - deg) * k
    Mx = Mx + torch.diag(diag)
    xs = torch.linalg.solve(Mx, torch.tensor(b))
    L = 0.5 * torch.sum((xs - torch.tensor(xt)) ** 2)
    L.backward()
    return float(L), th.grad.numpy()


def test_gradient_chain_matches_autograd_and_finite_differences():
    N = 4
    theta = si.theta_field(N**3)
    b = si.rhs_uniform(N**3)
    xt = si.x_target(N**3)
    A = si.stencil("7pt", N, np.exp(theta))
    M = si.to_scipy(A).toarray()
    x = np.linalg.solve(M, b)
    lam = np.linalg.solve(M, x - xt)          # adjoint solve (A symmetric)
    gval = oracle.csr_value_grad(A, lam, x)
    g = oracle.diffusion7_theta_grad(A, theta, gval)
    L, g_ref = _loss_and_grad_dense(N, theta, b, xt)
    assert np.abs(g - g_ref).max() <= 1e-10 * np.abs(g_ref).max()
    # central finite differences along a unit direction
    u = si.unit_direction(N**3)
    h = 1e-5

    def loss(th):
        Ah = si.stencil("7pt", N, np.exp(th))
        xh = np.linalg.solve(si.to_scipy(Ah).toarray(), b)
        return 0.5 * np.sum((xh - xt) ** 2)

    fd = (loss(theta + h * u) - loss(theta - h * u)) / (2 * h)
    assert abs(fd - g @ u) <= 1e-6 * abs(g @ u) + 1e-12


# ------------------------------------------------------ adaptive sweep count
def test_fgs_sweep_tol_stops_at_first_sweep_meeting_criterion():
    """With sweep_tol = d, each column takes the fewest sweeps (up to the cap)
    after which ||m - W a|| <= d ||m|| (the criterion of Sec. 3); d = 0 is
    the fixed-sweep FGS."""
    s = 8
    W = random_spd(s, seed=31, cond=30.0)
    B = np.random.default_rng(32).normal(size=(s, 3))
    X0, _ = oracle.fgs(W, B, 7)
    X0b, _ = oracle.fgs(W, B, 7, sweep_tol=0.0)
    assert np.array_equal(X0, X0b)
    for d in (1e-1, 1e-3, 1e-6):
        X, st = oracle.fgs(W, B, 500, sweep_tol=d)
        assert st == oracle.OK
        for c in range(3):
            m = B[:, c]
            res = lambda a: np.linalg.norm(m - W @ a)
            nu = next(v for v in range(1, 501)
                      if res(oracle.fgs(W, m, v)[0]) <= d * np.linalg.norm(m))
            assert np.array_equal(X[:, c], oracle.fgs(W, m, nu)[0])
            if nu > 1:
                assert res(oracle.fgs(W, m, nu - 1)[0]) > d * np.linalg.norm(m)
    # the cap still applies
    Xc, _ = oracle.fgs(W, B, 2, sweep_tol=1e-12)
    assert np.array_equal(Xc, oracle.fgs(W, B, 2)[0])


def test_sspcg_with_tight_sweep_tol_matches_cholesky():
    w = si.workload("poisson5", N=24)
    A, b = w["A"], w["b"]
    _, rc, hc = oracle.sspcg(A, b, s=4, sweeps=1, interval=w["interval"], tol=1e-10,
                             gram="cholesky", history=True)
    _, rf, hf = oracle.sspcg(A, b, s=4, sweeps=1000, interval=w["interval"], tol=1e-10,
                             sweep_tol=1e-13, history=True)
    assert rc["iters"] == rf["iters"]
    assert np.allclose(hf[:, 0], hc[:, 0], rtol=1e-6)


# ------------------------------------------------------------ monomial basis
def test_monomial_basis_is_matrix_powers_and_worse_conditioned():
    """basis = monomial: z_j = (M^{-1}A)^{j-1} M^{-1} r (the paper's
    introduction); its Gram matrix is far worse conditioned than the
    Chebyshev one (the reason for the Chebyshev basis)."""
    A = si.stencil("7pt", 8, np.exp(si.theta_field(512)))
    M = si.to_scipy(A).toarray()
    dinv = oracle.jacobi_inverse(A)
    r = np.random.default_rng(40).uniform(-1, 1, A.n)
    lo, hi = si.lanczos_bounds(A)
    s = 8
    Zm, Pm = oracle.mpk(A, dinv, r, s, (lo, hi), basis="monomial")
    v = dinv * r
    for j in range(s):
        assert np.abs(Zm[j] - v).max() <= 1e-12 * np.abs(v).max()
        v = dinv * (M @ v)
    Zc, Pc = oracle.mpk(A, dinv, r, s, (lo, hi))
    Wm, _ = oracle.gram(Zm, Pm[1:], Pm[0])
    Wc, _ = oracle.gram(Zc, Pc[1:], Pc[0])
    assert np.linalg.cond(Wm) > 1e3 * np.linalg.cond(Wc)


# ---------------------------------------------------------------- basis interval estimates


@pytest.mark.parametrize("kind,N", [("5pt", 10), ("7pt", 5), ("27pt", 4)])
def test_lanczos_full_run_reaches_closed_form_extremes(kind, N):
    # After n steps the extreme Ritz values are the extreme eigenvalues of
    # D^{-1}A (they converge first, loss of orthogonality notwithstanding).
    A = {"5pt": si.poisson5, "7pt": si.poisson7, "27pt": si.hpcg27}[kind](N)
    lo, hi, k = oracle.lanczos_bounds(A, si.start_vector(A.n), m=A.n)
    clo, chi = si.closed_form_bounds(kind, N)
    assert k == A.n
    assert abs(lo - clo) <= 1e-12 and abs(hi - chi) <= 1e-12


def test_lanczos_variable_coefficient_brackets_and_converges():
    N = 6
    A = si.stencil("27pt", N, si.coeff_blocks(N, block=2))
    d = 1.0 / oracle.jacobi_inverse(A)
    dense = si.to_scipy(A).toarray()
    ev = np.linalg.eigvalsh(dense / np.sqrt(np.outer(d, d)))
    v0 = si.start_vector(A.n)
    # Ritz values interlace: every m-step estimate lies inside the spectrum
    prev = (np.inf, -np.inf)
    for m in (2, 5, 10, 20):
        lo, hi, k = oracle.lanczos_bounds(A, v0, m)
        assert k == m
        assert ev[0] - 1e-12 <= lo and hi <= ev[-1] + 1e-12
        # and they move outwards as the Krylov space grows
        assert lo <= prev[0] + 1e-14 and hi >= prev[1] - 1e-14
        prev = (lo, hi)
    lo, hi, _ = oracle.lanczos_bounds(A, v0, A.n)
    assert abs(lo - ev[0]) <= 1e-10 * ev[-1] and abs(hi - ev[-1]) <= 1e-10 * ev[-1]


def test_lanczos_stops_on_invariant_start():
    # D^{-1}A = I when A is diagonal: every start vector spans an invariant
    # subspace.  With even powers of two on the diagonal and a scaled unit
    # start vector every product is exact, so the first beta is exactly 0.
    n = 40
    d = 4.0 ** np.arange(-5, n - 5)
    A = CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d, None)
    v0 = np.zeros(n)
    v0[7] = 3.0
    lo, hi, k = oracle.lanczos_bounds(A, v0, 20)
    assert (lo, hi, k) == (1.0, 1.0, 1)
    with pytest.raises(ValueError):
        oracle.lanczos_bounds(A, np.zeros(n), 20)


def test_lanczos_agrees_with_input_generator_estimate():
    # Two independent implementations of the same 20-step estimate.
    A = si.stencil("27pt", 12, si.coeff_blocks(12, block=4))
    lo, hi, _ = oracle.lanczos_bounds(A, si.start_vector(A.n), 20)
    ilo, ihi = si.lanczos_bounds(A)
    assert abs(lo - ilo) <= 1e-12 * ilo and abs(hi - ihi) <= 1e-12 * ihi


def test_power_method_monotone_and_converges_to_closed_form():
    # For constant coefficients M^{-1}A is symmetric; then the estimates
    # ||M^{-1}A v_l|| never decrease and stay below lambda_max.
    N = 10
    A = si.poisson5(N)
    chi = si.closed_form_bounds("5pt", N)[1]
    lo, hi, steps, hist = oracle.power_bounds(A, si.start_vector(A.n), rtol=1e-15, max_iter=5000)
    assert lo == 0.0 and steps < 5000
    assert np.all(np.diff(hist) >= -1e-15) and np.all(hist <= chi + 1e-14)
    assert abs(hi - chi) <= 1e-12


def test_power_method_stop_rule():
    A = si.stencil("27pt", 8, si.coeff_blocks(8, block=4))
    lo, hi, steps, hist = oracle.power_bounds(A, si.start_vector(A.n), rtol=1e-3, max_iter=50)
    assert steps == len(hist) and hist[-1] == hi
    rel = np.abs(np.diff(hist)) / hist[1:]
    # first step whose change is below rtol; none before it
    if steps < 50:
        assert rel[steps - 2] < 1e-3 and np.all(rel[:steps - 2] >= 1e-3)
    else:
        assert np.all(rel >= 1e-3)
    _, hi2, steps2, _ = oracle.power_bounds(A, si.start_vector(A.n), rtol=1e-3, max_iter=3)
    assert steps2 == min(3, steps) and hi2 == hist[steps2 - 1]


# ------------------------------------------------- one-ulp Gram perturbations
def test_gram_perturbations_are_one_ulp():
    """perturb_seed = 0 is the plain solve; with a seed every Gram entry moves
    by one unit in the last place: the iterates of an exact Gram solve stay
    within rounding of the plain ones, and the iteration counts of two FGS
    sweeps (rounding-driven) change with the seed."""
    w = si.workload("poisson5", N=64)
    A, b = w["A"], w["b"]
    kw = dict(s=4, interval=w["interval"], tol=1e-10)
    x0, r0 = oracle.sspcg(A, b, sweeps=2, **kw)
    xs, rs = oracle.sspcg(A, b, sweeps=2, perturb_seed=0, **kw)
    assert np.array_equal(x0, xs) and r0 == rs
    xc, rc = oracle.sspcg(A, b, sweeps=1, gram="cholesky", **kw)
    xp, rp = oracle.sspcg(A, b, sweeps=1, gram="cholesky", perturb_seed=7, **kw)
    assert not np.array_equal(xc, xp)
    assert np.linalg.norm(xp - xc) <= 1e-8 * np.linalg.norm(xc)
    assert abs(rp["iters"] - rc["iters"]) <= 1
    counts = {oracle.sspcg(A, b, sweeps=2, perturb_seed=k, **kw)[1]["iters"] for k in range(1, 9)}
    assert len(counts) >= 3
