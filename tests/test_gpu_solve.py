"""Solver-level parity of the HIP s-step PCG against the CPU oracle.

At small sweep counts (nu <= 3) the s-step iteration amplifies rounding
differences during the run (the Gram solves are inexact), so GPU and oracle
iterates separate in mid-run and meet again near the solution.  The checks
are therefore: the early trajectory (first 20 outer iterations) within
1e-10; solutions at a tight tolerance (relative residual 1e-12) within
1e-10; trajectory-stable settings (classical PCG, nu = 30, Cholesky Gram
solve) within 1e-10 at tolerance 1e-8.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_09790_amd as P
import sspcg_inputs as si
from spectral import kappa2
from spread import perturbed_counts, within_spread

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def gpu(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def poisson5():
    w = si.workload("poisson5")
    w["M"] = P.Matrix.from_csr(w["A"], fp32=True, device=DEV)
    return w


@pytest.fixture(scope="module")
def poisson7():
    w = si.workload("poisson7", N=24)
    w["M"] = P.Matrix.from_csr(w["A"], fp32=True, device=DEV)
    return w


@pytest.fixture(scope="module")
def diffusion27():
    N = 24
    A = si.stencil("27pt", N, si.coeff_blocks(N))
    w = dict(A=A, b=si.rhs_normal(A.n), interval=si.lanczos_bounds(A))
    w["M"] = P.Matrix.from_csr(A, fp32=True, device=DEV)
    return w


def run(w, **kw):
    x, info = P.solve(w["M"], gpu(w["b"]), interval=w["interval"], **kw)
    return x.cpu().numpy(), info


def test_early_trajectory_poisson5(poisson5):
    w = poisson5
    x, info = run(w, s=4, sweeps=2, tol=1e-30, max_outer=20)
    xo, ro = oracle.sspcg(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-30,
                          max_outer=20)
    assert info["status"] == P.NOT_CONVERGED and ro["status"] == oracle.NOT_CONVERGED
    assert info["outer_iters"] == 20
    assert rel(x, xo) <= 1e-10


@pytest.mark.parametrize("name", ["poisson5", "poisson7", "diffusion27"])
def test_tight_tolerance_solution(name, request):
    w = request.getfixturevalue(name)
    s = 6 if name == "diffusion27" else 4
    x, info = run(w, s=s, sweeps=2, tol=1e-12)
    xo, ro = oracle.sspcg(w["A"], w["b"], s=s, sweeps=2, interval=w["interval"], tol=1e-12)
    assert info["status"] == P.OK and ro["status"] == oracle.OK
    assert info["relres"] <= 1e-12
    assert rel(x, xo) <= 1e-10
    # the iteration count: within the rounding-only spread of the oracle
    counts = perturbed_counts(w["A"], w["b"], s=s, sweeps=2, interval=w["interval"], tol=1e-12,
                              runs=16 if name == "poisson5" else 6)
    print(f"{name}: device {info['outer_iters']} outer; perturbed oracle {counts.min()}.."
          f"{counts.max()} (mean {counts.mean():.1f})")
    assert within_spread(info["outer_iters"], counts)


@pytest.mark.parametrize("s", [2, 4, 6, 8])
@pytest.mark.parametrize("sweeps", [1, 2, 3])
def test_s_nu_grid(poisson7, s, sweeps):
    w = poisson7
    x, info = run(w, s=s, sweeps=sweeps, tol=1e-12)
    xo, ro = oracle.sspcg(w["A"], w["b"], s=s, sweeps=sweeps, interval=w["interval"], tol=1e-12)
    assert info["status"] == ro["status"] == 0
    assert rel(x, xo) <= 1e-10


@pytest.mark.parametrize("gram,sweeps", [("fgs", 30), ("cholesky", 1)])
def test_trajectory_stable_settings(poisson5, gram, sweeps):
    w = poisson5
    x, info = run(w, s=4, sweeps=sweeps, gram=gram, tol=1e-8, history=True)
    xo, ro, ho = oracle.sspcg(w["A"], w["b"], s=4, sweeps=sweeps, interval=w["interval"],
                              tol=1e-8, gram=gram, history=True)
    assert info["outer_iters"] == ro["iters"]
    assert rel(x, xo) <= 1e-10
    h = info["history"]
    assert np.abs(h[:, 0] - ho[:, 0]).max() <= 1e-9 * ho[0, 0]


def test_history_matches_oracle_early(poisson7):
    w = poisson7
    _, info = run(w, s=4, sweeps=2, tol=1e-30, max_outer=10, history=True)
    _, _, ho = oracle.sspcg(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-30,
                            max_outer=10, history=True)
    h = info["history"]
    assert h.shape == (10, 4) and ho.shape == (10, 4)
    assert np.allclose(h[:, 0], ho[:, 0], rtol=1e-9, atol=0)
    assert np.allclose(h[:, 1], ho[:, 1], rtol=1e-6, atol=1e-12)
    assert np.allclose(h[:-1, 2], ho[:-1, 2], rtol=1e-6, atol=1e-12)
    # conjugacy defect ||B2 - W beta||_F = ||Q_{k+1}^T A Q_k||_F (Sec. 2)
    assert np.allclose(h[:-1, 3], ho[:-1, 3], rtol=1e-6, atol=0)
    assert np.all(h[:-1, 3] > 0)


@pytest.mark.parametrize("name", ["poisson5", "diffusion27"])
def test_classical_pcg(name, request):
    w = request.getfixturevalue(name)
    x, info = P.pcg(w["M"], gpu(w["b"]), tol=1e-8, history=True)
    xo, ro, ho = oracle.pcg(w["A"], w["b"], tol=1e-8, history=True)
    assert info["status"] == P.OK
    assert abs(info["outer_iters"] - ro["iters"]) <= 1
    assert rel(x.cpu().numpy(), xo) <= 1e-10
    k = min(len(ho), len(info["history"])) - 2
    assert np.allclose(info["history"][:k], ho[:k], rtol=1e-8)


def test_s1_is_classical_pcg(poisson5):
    w = poisson5
    x1, i1 = run(w, s=1, sweeps=3, tol=1e-8)
    x2, i2 = P.pcg(w["M"], gpu(w["b"]), tol=1e-8)
    assert abs(i1["outer_iters"] - i2["outer_iters"]) <= 1
    assert rel(x1, x2.cpu().numpy()) <= 1e-9


def test_deterministic(diffusion27):
    w = diffusion27
    x1, i1 = run(w, s=6, sweeps=2, tol=1e-8)
    x2, i2 = run(w, s=6, sweeps=2, tol=1e-8)
    assert i1["outer_iters"] == i2["outer_iters"]
    assert np.array_equal(x1, x2)


@pytest.mark.parametrize("name", ["poisson7", "diffusion27"])
def test_mixed_precision_refinement(name, request):
    w = request.getfixturevalue(name)
    x, info = run(w, s=4, sweeps=2, tol=1e-10, precision="mixed", history=True)
    assert info["status"] == P.OK and info["relres"] <= 1e-10
    assert 1 <= info["refinements"] <= 8
    h = info["history"]
    assert h[-1] <= 1e-10 and np.all(np.diff(h) < 0)
    # true residual recomputed independently
    r = w["b"] - oracle.spmv(w["A"], x)
    assert np.linalg.norm(r) <= 1.0001e-10 * np.linalg.norm(w["b"])
    # error against x_ref, the oracle's classical PCG to 1e-13: reported, and
    # within the forward-error bound kappa_2(A) ||b - A x|| / ||b||
    xo, ro = oracle.pcg(w["A"], w["b"], tol=1e-13)
    err = rel(x, xo)
    bound = kappa2(w["A"]) * np.linalg.norm(r) / np.linalg.norm(w["b"])
    print(f"{name}: mixed vs x_ref relative error {err:.2e} (bound {bound:.2e}), "
          f"{info['refinements']} refinements, {info['outer_iters']} inner iterations")
    assert err <= bound
    xm, rm = oracle.sspcg_mixed(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-10)
    assert rm["status"] == oracle.OK
    assert abs(rm["refinements"] - info["refinements"]) <= 2


def test_mixed_needs_fp32_values(poisson5):
    M = P.Matrix.from_csr(poisson5["A"], device=DEV)
    with pytest.raises(P.SSPCGError) as e:
        P.solve(M, gpu(poisson5["b"]), interval=poisson5["interval"], precision="mixed")
    assert e.value.status == P.ERR_UNSUPPORTED


# ------------------------------------------------------------------ edge cases
def test_zero_rhs_gives_zero(poisson5):
    x, info = P.solve(poisson5["M"], torch.zeros(4096, dtype=torch.float64, device=DEV),
                      x0=torch.ones(4096, dtype=torch.float64, device=DEV),
                      interval=poisson5["interval"])
    assert info["status"] == P.OK and info["outer_iters"] == 0
    assert torch.count_nonzero(x).item() == 0


def test_exact_start_takes_no_iteration(poisson5):
    w = poisson5
    xs, _ = oracle.pcg(w["A"], w["b"], tol=1e-14)
    x, info = P.solve(w["M"], gpu(w["b"]), x0=gpu(xs), interval=w["interval"], tol=1e-8)
    assert info["status"] == P.OK and info["outer_iters"] == 0
    assert np.array_equal(x.cpu().numpy(), xs)


def test_nonfinite_rhs(poisson5):
    b = poisson5["b"].copy()
    b[17] = np.nan
    _, info = P.solve(poisson5["M"], gpu(b), interval=poisson5["interval"], raise_on_error=False)
    assert info["status"] == P.ERR_NONFINITE


def test_iteration_limit(poisson5):
    x, info = run(poisson5, s=4, sweeps=2, tol=1e-8, max_outer=1)
    assert info["status"] == P.NOT_CONVERGED and info["outer_iters"] == 1
    xo, ro = oracle.sspcg(poisson5["A"], poisson5["b"], s=4, sweeps=2,
                          interval=poisson5["interval"], tol=1e-8, max_outer=1)
    assert rel(x, xo) <= 1e-12


@pytest.mark.parametrize("shift,s", [(0.5, 2), (0.5, 4), (1.0, 2)])
def test_breakdown_returns_last_iterate(shift, s):
    """A symmetric indefinite matrix (positive diagonal): the Gram solve
    breaks down after a few outer iterations, as in the oracle, and x is the
    oracle's last iterate there (including the x update that the solve
    defers to the next block update)."""
    A = si.poisson5(16)
    d = A.col == np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    val = A.val.copy()
    val[d] -= shift
    B = si.CSR(A.n, A.row_ptr, A.col, val, A.shape3)
    b = si.rhs_uniform(A.n)
    xo, ro = oracle.sspcg(B, b, s=s, sweeps=2, interval=(0.05, 8.0), tol=1e-10, max_outer=200)
    assert ro["status"] == oracle.BREAKDOWN and ro["iters"] >= 1
    M = P.Matrix.from_csr(B, device=DEV)
    x, info = P.solve(M, gpu(b), s=s, sweeps=2, interval=(0.05, 8.0), tol=1e-10, max_outer=200,
                      raise_on_error=False)
    assert info["status"] == P.ERR_BREAKDOWN and info["outer_iters"] == ro["iters"]
    assert rel(x.cpu().numpy(), xo) <= 1e-10


@pytest.mark.parametrize("kind,N,s", [("5pt", 3, 2), ("5pt", 9, 16), ("7pt", 5, 3),
                                      ("27pt", 4, 5)])
def test_small_and_ragged_systems(kind, N, s):
    A = si.stencil(kind, N)
    b = si.rhs_uniform(A.n)
    lo, hi = si.closed_form_bounds(kind, N)
    M = P.Matrix.from_csr(A, device=DEV)
    x, info = P.solve(M, gpu(b), s=s, sweeps=8, interval=(lo * 0.99, hi * 1.01), tol=1e-11)
    xo, ro = oracle.sspcg(A, b, s=s, sweeps=8, interval=(lo * 0.99, hi * 1.01), tol=1e-11)
    assert info["status"] == ro["status"] == 0
    assert rel(x.cpu().numpy(), xo) <= 1e-9


def test_workspace_too_small(poisson5):
    import ctypes
    from paper_2603_09790_amd import _lib as L
    p = L.Params()
    L.lib().sspcg_default_params(ctypes.byref(p))
    p.lambda_max = 2.0
    b = gpu(poisson5["b"])
    x = torch.zeros_like(b)
    work = torch.empty(1024, dtype=torch.uint8, device=DEV)
    poll = torch.empty(L.POLL_BYTES, dtype=torch.uint8, pin_memory=True)
    res = L.Result()
    args = (poisson5["M"].handle, ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(x.data_ptr()),
            ctypes.byref(p), ctypes.c_void_p(work.data_ptr()), 1024)
    st = L.lib().sspcg_solve(*args, ctypes.c_void_p(poll.data_ptr()), None, ctypes.byref(res),
                             None, None)
    assert st == L.ERR_WORKSPACE and res.status == L.ERR_WORKSPACE
    # the poll buffer is checked before the workspace size
    st = L.lib().sspcg_solve(*args, None, None, ctypes.byref(res), None, None)
    assert st == L.ERR_ARG


# ------------------------------------------------------------ differentiation
def test_diffusion_solve_gradient():
    N = 8
    theta = si.theta_field(N**3)
    A = si.stencil("7pt", N, np.exp(theta))
    b = si.rhs_uniform(A.n)
    xt = si.x_target(A.n)
    interval = si.lanczos_bounds(A)
    M = P.Matrix.from_csr(A, device=DEV)
    opts = dict(s=4, sweeps=2, interval=interval, tol=1e-14)
    th = gpu(theta).requires_grad_(True)
    x = P.DiffusionSolve.apply(th, gpu(b), M, opts)
    loss = 0.5 * torch.sum((x - gpu(xt)) ** 2)
    loss.backward()
    g = th.grad.cpu().numpy()
    # oracle chain: solve, adjoint solve, value gradient, theta gradient;
    # both sides solve to 1e-14
    xo, _ = oracle.sspcg(A, b, s=4, sweeps=2, interval=interval, tol=1e-14)
    lam, _ = oracle.sspcg(A, xo - xt, s=4, sweeps=2, interval=interval, tol=1e-14)
    go = oracle.diffusion7_theta_grad(A, theta, oracle.csr_value_grad(A, lam, xo))
    print(f"8^3 gradient vs oracle: {rel(g, go):.2e}")
    assert rel(g, go) <= 1e-10
    # central finite differences of the loss along a unit direction
    u = si.unit_direction(A.n)
    h = 1e-5

    def loss_at(t):
        Ah = si.stencil("7pt", N, np.exp(t))
        xh, _ = oracle.sspcg(Ah, b, s=4, sweeps=2, interval=interval, tol=1e-14)
        return 0.5 * np.sum((xh - xt) ** 2)

    fd = (loss_at(theta + h * u) - loss_at(theta - h * u)) / (2 * h)
    assert abs(fd - g @ u) <= 1e-6 * abs(g @ u)


def test_sparse_solve_value_and_rhs_gradient():
    N = 6
    A = si.stencil("7pt", N, np.exp(si.theta_field(N**3)))
    b = si.rhs_uniform(A.n)
    interval = si.lanczos_bounds(A)
    M = P.Matrix.from_csr(A, device=DEV)
    val = gpu(A.val).requires_grad_(True)
    bb = gpu(b).requires_grad_(True)
    x = P.SparseSolve.apply(val, bb, M, dict(s=3, sweeps=3, interval=interval, tol=1e-13))
    w = torch.linspace(-1, 1, A.n, dtype=torch.float64, device=DEV)
    (x * w).sum().backward()
    D = si.to_scipy(A).toarray()
    lam = np.linalg.solve(D, w.cpu().numpy())
    xs = np.linalg.solve(D, b)
    assert rel(bb.grad.cpu().numpy(), lam) <= 1e-9
    rows = np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    assert rel(val.grad.cpu().numpy(), -lam[rows] * xs[A.col]) <= 1e-9


@pytest.mark.parametrize("sweep_tol", [1e-2, 1e-6])
def test_adaptive_sweeps(poisson5, sweep_tol):
    w = poisson5
    x, info = run(w, s=4, sweeps=200, sweep_tol=sweep_tol, tol=1e-8, history=True)
    xo, ro, ho = oracle.sspcg(w["A"], w["b"], s=4, sweeps=200, interval=w["interval"], tol=1e-8,
                              sweep_tol=sweep_tol, history=True)
    assert info["status"] == ro["status"] == 0
    assert abs(info["outer_iters"] - ro["iters"]) <= 2
    assert rel(x, xo) <= 1e-8
    # the reduced systems meet the criterion (or the sweep cap was reached)
    assert np.all(info["history"][:, 1] <= sweep_tol * (1 + 1e-6))


def test_warm_restart_from_stopped_solve(poisson7):
    """The solver's state is x: a solve stopped at its iteration limit and
    restarted from its x converges to the same solution (a new Krylov basis,
    so not the same trajectory)."""
    w = poisson7
    x1, i1 = run(w, s=4, sweeps=2, tol=1e-10, max_outer=40)
    assert i1["status"] == P.NOT_CONVERGED and i1["outer_iters"] == 40
    x2, i2 = P.solve(w["M"], gpu(w["b"]), x0=gpu(x1), s=4, sweeps=2, interval=w["interval"],
                     tol=1e-10)
    assert i2["status"] == P.OK
    xs, _ = oracle.pcg(w["A"], w["b"], tol=1e-13)
    assert rel(x2.cpu().numpy(), xs) <= 1e-7


def test_debug_sync_mode():
    """SSPCG_DEBUG_SYNC=1 (read once per process) synchronizes after every
    launch; a solve in a child process with it set gives the same result."""
    import os
    import subprocess
    import sys
    code = (
        "import numpy as np, torch, paper_2603_09790_amd as P, sspcg_inputs as si\n"
        "w = si.workload('poisson5', N=32)\n"
        "M = P.Matrix.from_csr(w['A'], device='cuda:0')\n"
        "x, i = P.solve(M, torch.from_numpy(w['b']), s=4, sweeps=2, interval=w['interval'],"
        " tol=1e-10)\n"
        "np.save('/tmp/sspcg_debug_sync_x.npy', x.cpu().numpy())\n"
        "print(i['status'], i['outer_iters'])\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SSPCG_DEBUG_SYNC="1", PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=240, cwd=root)
    assert out.returncode == 0, out.stderr[-2000:]
    st, iters = map(int, out.stdout.split()[-2:])
    w = si.workload("poisson5", N=32)
    M = P.Matrix.from_csr(w["A"], device=DEV)
    x, info = P.solve(M, gpu(w["b"]), s=4, sweeps=2, interval=w["interval"], tol=1e-10)
    assert st == 0 and iters == info["outer_iters"]
    assert np.array_equal(np.load("/tmp/sspcg_debug_sync_x.npy"), x.cpu().numpy())


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_results_do_not_depend_on_the_grid(precision):
    """Reductions write one partial per virtual block, a count fixed by the
    problem size: a solve whose persistent grids are capped at one workgroup
    per CU (SSPCG_GRID_BLOCKS_PER_CU=1, in a child process; 256 workgroups
    for 512 virtual blocks at 64^3) gives the same iterates bit for bit as the
    default grids."""
    import os
    import subprocess
    import sys
    out_path = f"/tmp/sspcg_grid_x_{precision}.npy"
    code = (
        "import numpy as np, torch, paper_2603_09790_amd as P, sspcg_inputs as si\n"
        "A = si.stencil('27pt', 64, si.coeff_blocks(64))\n"
        "M = P.Matrix.from_csr(A, fp32=True, device='cuda:0')\n"
        "b = torch.from_numpy(si.rhs_normal(A.n))\n"
        f"x, i = P.solve(M, b, s=6, sweeps=2, interval=si.lanczos_bounds(A), tol=1e-10, "
        f"precision='{precision}')\n"
        f"np.save('{out_path}', x.cpu().numpy())\n"
        "print(i['status'], i['outer_iters'])\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, SSPCG_GRID_BLOCKS_PER_CU="1", PYTHONPATH=root)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         timeout=240, cwd=root)
    assert out.returncode == 0, out.stderr[-2000:]
    st, iters = map(int, out.stdout.split()[-2:])
    A = si.stencil("27pt", 64, si.coeff_blocks(64))
    M = P.Matrix.from_csr(A, fp32=True, device=DEV)
    x, info = P.solve(M, gpu(si.rhs_normal(A.n)), s=6, sweeps=2, interval=si.lanczos_bounds(A),
                      tol=1e-10, precision=precision)
    assert st == 0 and iters == info["outer_iters"]
    assert np.array_equal(np.load(out_path), x.cpu().numpy())


def test_monomial_basis_solve(poisson7):
    w = poisson7
    x, info = run(w, s=4, sweeps=2, basis="monomial", tol=1e-30, max_outer=10)
    xo, ro = oracle.sspcg(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-30,
                          max_outer=10, basis="monomial")
    assert info["outer_iters"] == ro["iters"] == 10
    assert rel(x, xo) <= 1e-9


def test_diffusion_gradient_32cube_finite_differences_and_oracle():
    """The differentiable form's check instance: 7-point diffusion on 32^3,
    theta ~ N(0, 0.5^2), loss 0.5 ||x - x_target||^2.  Gradient against
    central differences (GPU solves at 1e-14) and the oracle's gradient chain
    (both sides at 1e-14).

    The loss is ~1.7e4 and the solves carry ~1e-13 relative noise, so the
    difference quotient uses a direction with O(1) entries per cell, the
    fourth-order central stencil with h = 2e-3 (truncation ~h^4) and loss
    differences formed without cancellation: L(a) - L(b) =
    0.5 (x_a - x_b)^T (x_a + x_b - 2 x_target).  With the oracle's solves this
    reaches ~1e-8 relative; a unit direction at h = 1e-4 only ~1e-4."""
    N = 32
    w = si.workload("diffusion7", N=N)
    A, theta, b, xt = w["A"], w["theta"], w["b"], w["x_target"]
    interval = w["interval"]
    M = P.Matrix.from_csr(A, device=DEV)
    opts = dict(s=4, sweeps=2, interval=interval, tol=1e-14)
    th = gpu(theta).requires_grad_(True)
    x = P.DiffusionSolve.apply(th, gpu(b), M, opts)
    loss = 0.5 * torch.sum((x - gpu(xt)) ** 2)
    loss.backward()
    g = th.grad.cpu().numpy()
    u = si.unit_direction(A.n) * np.sqrt(A.n)
    h = 2e-3

    def x_at(t):
        return P.DiffusionSolve.apply(gpu(t), gpu(b), M, opts).cpu().numpy()

    def dloss(t1, t2):
        x1, x2 = x_at(t1), x_at(t2)
        return 0.5 * (x1 - x2) @ (x1 + x2 - 2 * xt)

    d1 = dloss(theta + h * u, theta - h * u)
    d2 = dloss(theta + 2 * h * u, theta - 2 * h * u)
    fd = (8 * d1 - d2) / (12 * h)
    print(f"32^3 gradient vs finite differences: {abs(fd - g @ u) / abs(g @ u):.2e}")
    assert abs(fd - g @ u) <= 1e-6 * abs(g @ u)
    xo, _ = oracle.sspcg(A, b, s=4, sweeps=2, interval=interval, tol=1e-14)
    lam, _ = oracle.sspcg(A, xo - xt, s=4, sweeps=2, interval=interval, tol=1e-14)
    go = oracle.diffusion7_theta_grad(A, theta, oracle.csr_value_grad(A, lam, xo))
    print(f"32^3 gradient vs oracle: {rel(g, go):.2e}")
    assert rel(g, go) <= 1e-10


@pytest.mark.parametrize("check_every", [1, 8])
def test_graph_replay_matches_eager(poisson5, check_every):
    """use_graph: a batch of outer iterations captured once into a HIP graph
    and replayed.  Several graph solves, with eager solves and syncs between
    them, each equal the eager result bit for bit (same kernels, same order)."""
    w = poisson5
    s_ = torch.cuda.Stream()
    b = gpu(w["b"])
    with torch.cuda.stream(s_):
        xe, ie = P.solve(w["M"], b, s=4, sweeps=2, interval=w["interval"], tol=1e-10,
                         check_every=check_every)
        for _ in range(3):
            xg, ig = P.solve(w["M"], b, s=4, sweeps=2, interval=w["interval"], tol=1e-10,
                             check_every=check_every, graph=True)
            torch.cuda.synchronize()
            xe2, _ = P.solve(w["M"], b, s=4, sweeps=2, interval=w["interval"], tol=1e-10,
                             check_every=check_every)
            torch.cuda.synchronize()
            assert ig["status"] == P.OK and ig["outer_iters"] == ie["outer_iters"]
            assert torch.equal(xg, xe) and torch.equal(xe2, xe)
    # the iteration limit is respected in graph mode too, and the iterate
    # left there (with its last x update applied after the loop) is the
    # eager solve's
    with torch.cuda.stream(s_):
        xl, il = P.solve(w["M"], b, s=4, sweeps=2, interval=w["interval"], tol=1e-10,
                         max_outer=13, check_every=8, graph=True)
        xle, ile = P.solve(w["M"], b, s=4, sweeps=2, interval=w["interval"], tol=1e-10,
                           max_outer=13, check_every=8)
    torch.cuda.synchronize()
    assert il["status"] == P.NOT_CONVERGED and il["outer_iters"] == 13
    assert ile["outer_iters"] == 13 and torch.equal(xl, xle)


def test_two_solves_on_one_matrix_at_once():
    """Solves only read the matrix handle: two solves on one matrix, each with
    its own workspace and poll buffer, run at once from two host threads on
    two streams through the C ABI and return the same bits as the same solves
    run one after the other (the reductions have a fixed order, so running
    beside another solve changes nothing)."""
    import ctypes
    from concurrent.futures import ThreadPoolExecutor
    from paper_2603_09790_amd import _lib as L
    from paper_2603_09790_amd import solver as S
    w = si.workload("diffusion27", N=40)
    A = w["A"]
    M = P.Matrix.from_csr(A, device=DEV)
    bs = [gpu(w["b"]), gpu(si.rhs_uniform(A.n))]
    opts = dict(s=6, sweeps=2, interval=w["interval"], tol=1e-10)
    refs = [P.solve(M, b, **opts) for b in bs]
    p = S._params(6, 2, w["interval"], 1e-10, "fp64", "fgs", 20000, 1e-4, 20, 8)
    nbytes = ctypes.c_size_t()
    assert L.lib().sspcg_workspace_bytes(M.handle, ctypes.byref(p), ctypes.byref(nbytes)) == L.OK
    works = [torch.empty(nbytes.value, dtype=torch.uint8, device=DEV) for _ in bs]
    polls = [torch.empty(L.POLL_BYTES, dtype=torch.uint8, pin_memory=True) for _ in bs]
    xs = [torch.zeros(A.n, dtype=torch.float64, device=DEV) for _ in bs]
    streams = [torch.cuda.Stream(device=DEV) for _ in bs]
    torch.cuda.synchronize()

    def run(i):
        res = L.Result()
        st = L.lib().sspcg_solve(M.handle, ctypes.c_void_p(bs[i].data_ptr()),
                                 ctypes.c_void_p(xs[i].data_ptr()), ctypes.byref(p),
                                 ctypes.c_void_p(works[i].data_ptr()), nbytes.value,
                                 ctypes.c_void_p(polls[i].data_ptr()),
                                 ctypes.c_void_p(streams[i].cuda_stream), ctypes.byref(res),
                                 None, None)
        return st, res.outer_iters

    with ThreadPoolExecutor(2) as ex:
        out = list(ex.map(run, range(2)))
    torch.cuda.synchronize()
    for (st, iters), (xr, ir), x in zip(out, refs, xs):
        assert st == L.OK and iters == ir["outer_iters"]
        assert torch.equal(x, xr)
