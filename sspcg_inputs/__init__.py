"""Seeded synthetic inputs for the s-step PCG solver and its CPU oracle.

This package builds the test systems: stencil matrices in CSR form,
coefficient fields, right-hand sides and the spectral intervals that scale
the Chebyshev basis.  It is the only code shared by the HIP path's tests and
the oracle, and it holds none of the solver's arithmetic: no Krylov basis, no
Gram reduction, no Gauss-Seidel sweep, no search-direction update.

Conventions (the paper's experiments use the 27-point Poisson matrix of the
HPCG benchmark with Dirichlet boundaries, Sec. "Performance Results at Large
Scale"; the variable-coefficient forms generalise it):

* Unknowns are ordered lexicographically, x fastest:
  ``idx = x + Nx*(y + Ny*z)``.  Column indices inside a row are sorted and
  the diagonal is stored explicitly.
* No 1/h^2 factor: the Jacobi preconditioner makes M^{-1}A scale-free.
* Variable coefficients: for every in-domain neighbour j of cell i the
  off-diagonal entry is ``-w_ij`` with the harmonic mean
  ``w_ij = 2*k_i*k_j/(k_i+k_j)``; the diagonal is ``sum_j w_ij`` plus one
  ``k_i`` per stencil neighbour that falls outside the domain (a Dirichlet
  ghost cell carrying the cell's own coefficient).  With ``k == 1`` this is
  exactly the constant-coefficient stencil (diagonal 4, 6 or 26, off-diagonal
  -1).
* Random numbers come from numpy's PCG64 ``default_rng(seed)``.  Seeds used
  by the standard workloads: right-hand side 0, coefficient field 1,
  Lanczos start vector 2, log-coefficients theta 3, regression target 4,
  finite-difference direction 5, sampled solution indices 6, probe vectors 7.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "CSR", "offsets", "stencil", "stencil_numpy", "poisson5", "poisson7", "hpcg27",
    "coeff_blocks", "theta_field", "rhs_uniform", "rhs_normal",
    "x_target", "unit_direction", "closed_form_bounds", "start_vector", "lanczos_bounds",
    "power_bounds", "nnz_formula", "jacobi_inverse", "to_scipy",
    "workload", "sample_indices", "probe_vectors", "digest",
]

SEED_RHS = 0
SEED_COEFF = 1
SEED_LANCZOS = 2
SEED_THETA = 3
SEED_TARGET = 4
SEED_DIRECTION = 5
SEED_SAMPLES = 6
SEED_PROBES = 7


@dataclass
class CSR:
    """A square CSR matrix with int32 indices and float64 values."""
    n: int
    row_ptr: np.ndarray   # int32[n+1]
    col: np.ndarray       # int32[nnz]
    val: np.ndarray       # float64[nnz]
    shape3: tuple         # (Nz, Ny, Nx) of the grid the matrix lives on

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])


def offsets(kind: str) -> list:
    """Stencil offsets (dz, dy, dx) sorted by linear offset, centre included."""
    if kind == "5pt":
        offs = [(0, -1, 0), (0, 0, -1), (0, 0, 0), (0, 0, 1), (0, 1, 0)]
    elif kind == "7pt":
        offs = [(-1, 0, 0), (0, -1, 0), (0, 0, -1), (0, 0, 0),
                (0, 0, 1), (0, 1, 0), (1, 0, 0)]
    elif kind == "27pt":
        offs = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1)
                for dx in (-1, 0, 1)]
    else:
        raise ValueError(f"unknown stencil kind {kind!r}")
    return offs


def _grid(kind: str, N: int) -> tuple:
    return (1, N, N) if kind == "5pt" else (N, N, N)


def stencil(kind: str, N: int, kappa: np.ndarray | None = None) -> CSR:
    """Assemble the (variable-coefficient) stencil matrix on an N^d grid.

    ``kappa`` is a per-cell coefficient array of length n (None means 1).
    Uses the C assembler in stencil.c; ``stencil_numpy`` is the same
    definition written with array operations and serves as its check.
    """
    from . import _native
    Nz, Ny, Nx = _grid(kind, N)
    if min(Nx, Ny) < 3 or (Nz != 1 and Nz < 3):
        raise ValueError("grid must be at least 3 cells wide")
    n = Nz * Ny * Nx
    offs = np.ascontiguousarray(np.array(offsets(kind), dtype=np.int32).reshape(-1))
    K = len(offs) // 3
    kap = None
    if kappa is not None:
        kap = np.ascontiguousarray(kappa, dtype=np.float64)
        if kap.shape != (n,):
            raise ValueError("kappa must have one entry per cell")
    L = _native.lib()
    nnz = L.inp_stencil_nnz(Nz, Ny, Nx, K, offs.ctypes.data)
    if nnz < 0 or nnz >= 2**31:
        raise ValueError("bad grid or nnz exceeds int32 range")
    row_ptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz, dtype=np.float64)
    rc = L.inp_stencil(Nz, Ny, Nx, K, offs.ctypes.data,
                       None if kap is None else kap.ctypes.data,
                       row_ptr.ctypes.data, col.ctypes.data, val.ctypes.data)
    if rc != 0:
        raise RuntimeError("stencil assembly failed")
    return CSR(n, row_ptr, col, val, (Nz, Ny, Nx))


def stencil_numpy(kind: str, N: int, kappa: np.ndarray | None = None) -> CSR:
    """Array-operation version of ``stencil`` (slow on large grids)."""
    Nz, Ny, Nx = _grid(kind, N)
    if min(Nx, Ny) < 3 or (Nz != 1 and Nz < 3):
        raise ValueError("grid must be at least 3 cells wide")
    n = Nz * Ny * Nx
    offs = offsets(kind)
    K = len(offs)
    idx = np.arange(n, dtype=np.int64)
    x = idx % Nx
    y = (idx // Nx) % Ny
    z = idx // (Nx * Ny)
    ki = None if kappa is None else np.ascontiguousarray(kappa, dtype=np.float64)
    if ki is not None and ki.shape != (n,):
        raise ValueError("kappa must have one entry per cell")

    valid = np.empty((n, K), dtype=bool)
    cols = np.empty((n, K), dtype=np.int32)
    vals = np.zeros((n, K), dtype=np.float64)
    diag = np.zeros(n, dtype=np.float64)
    nvalid_nb = np.zeros(n, dtype=np.int32)
    centre = None
    for k, (dz, dy, dx) in enumerate(offs):
        ok = ((x + dx >= 0) & (x + dx < Nx) & (y + dy >= 0) & (y + dy < Ny)
              & (z + dz >= 0) & (z + dz < Nz))
        lin = dx + Nx * (dy + Ny * dz)
        valid[:, k] = ok
        j = np.where(ok, idx + lin, idx)
        cols[:, k] = j
        if (dz, dy, dx) == (0, 0, 0):
            centre = k
            continue
        if ki is None:
            w = np.where(ok, 1.0, 0.0)
        else:
            kj = ki[j]
            w = np.where(ok, 2.0 * ki * kj / (ki + kj), 0.0)
        vals[:, k] = -w
        diag += w
        nvalid_nb += ok
        del ok, j, w
    nmiss = (K - 1) - nvalid_nb
    diag += nmiss * (1.0 if ki is None else ki)
    vals[:, centre] = diag
    del diag, nmiss, nvalid_nb, x, y, z, idx

    counts = valid.sum(axis=1, dtype=np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 range")
    m = valid.ravel()
    col = cols.ravel()[m]
    del cols
    val = vals.ravel()[m]
    del vals, valid, m
    return CSR(n, row_ptr.astype(np.int32), col, val, (Nz, Ny, Nx))


def poisson5(N: int) -> CSR:
    """2D 5-point Poisson matrix on N x N (diagonal 4, off-diagonal -1)."""
    return stencil("5pt", N)


def poisson7(N: int) -> CSR:
    """3D 7-point Poisson matrix on N^3 (diagonal 6, off-diagonal -1)."""
    return stencil("7pt", N)


def hpcg27(N: int) -> CSR:
    """3D 27-point matrix as in HPCG on N^3 (diagonal 26, off-diagonal -1)."""
    return stencil("27pt", N)


def nnz_formula(kind: str, N: int) -> int:
    """Closed-form nonzero count of the Dirichlet stencil matrices."""
    if kind == "5pt":
        return 5 * N * N - 4 * N
    if kind == "7pt":
        return 7 * N**3 - 6 * N**2
    if kind == "27pt":
        return (3 * N - 2) ** 3
    raise ValueError(kind)


def coeff_blocks(N: int, block: int = 8, log10_lo: float = -2.0,
                 log10_hi: float = 2.0, seed: int = SEED_COEFF) -> np.ndarray:
    """Piecewise-constant coefficients on block^3 cubes, log10 k ~ U[lo, hi]."""
    if N % block:
        raise ValueError("N must be a multiple of the block size")
    nb = N // block
    rng = np.random.default_rng(seed)
    logk = rng.uniform(log10_lo, log10_hi, size=(nb, nb, nb))
    kb = np.power(10.0, logk)
    k = np.repeat(np.repeat(np.repeat(kb, block, axis=0), block, axis=1),
                  block, axis=2)
    return np.ascontiguousarray(k.reshape(-1))


def theta_field(n: int, sigma: float = 0.5, seed: int = SEED_THETA) -> np.ndarray:
    """Per-cell log-coefficients theta ~ N(0, sigma^2)."""
    return np.random.default_rng(seed).normal(0.0, sigma, size=n)


def rhs_uniform(n: int, seed: int = SEED_RHS) -> np.ndarray:
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def rhs_normal(n: int, seed: int = SEED_RHS) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, 1.0, size=n)


def x_target(n: int, seed: int = SEED_TARGET) -> np.ndarray:
    return np.random.default_rng(seed).normal(0.0, 1.0, size=n)


def unit_direction(n: int, seed: int = SEED_DIRECTION) -> np.ndarray:
    v = np.random.default_rng(seed).normal(0.0, 1.0, size=n)
    return v / np.linalg.norm(v)


def sample_indices(n: int, m: int, seed: int = SEED_SAMPLES) -> np.ndarray:
    """m distinct row indices in [0, n), sorted (where a solution is sampled)."""
    m = min(m, n)
    idx = np.random.default_rng(seed).choice(n, size=m, replace=False)
    return np.sort(idx).astype(np.int64)


def probe_vectors(n: int, k: int, seed: int = SEED_PROBES) -> np.ndarray:
    """k vectors with N(0,1) entries, shape (k, n): a solution is summarised
    by its inner products with them."""
    return np.random.default_rng(seed).normal(0.0, 1.0, size=(k, n))


def digest(*arrays) -> str:
    """SHA-1 of the bytes of the arrays, to tell whether two machines built
    the same inputs."""
    import hashlib
    h = hashlib.sha1()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def jacobi_inverse(A: CSR) -> np.ndarray:
    """1/diag(A) (used by the interval estimators only)."""
    from . import _native
    d = np.empty(A.n)
    _native.lib().inp_diagonal(A.n, A.row_ptr.ctypes.data, A.col.ctypes.data,
                               A.val.ctypes.data, d.ctypes.data)
    return 1.0 / d


def to_scipy(A: CSR):
    import scipy.sparse as sp
    return sp.csr_matrix((A.val, A.col, A.row_ptr), shape=(A.n, A.n))


def closed_form_bounds(kind: str, N: int) -> tuple:
    """Extreme eigenvalues of D^{-1}A for the constant-coefficient stencils.

    The Dirichlet stencils are sums of Kronecker products of the 1D matrices
    tridiag(1, 1, 1) (27-point) or tridiag(-1, 2, -1) (5/7-point), whose
    eigenvalues use theta_k = k*pi/(N+1), k = 1..N:
      5-point : 1 - (cos th_i + cos th_j)/2
      7-point : 1 - (cos th_i + cos th_j + cos th_k)/3
      27-point: (27 - prod_d (1 + 2 cos th_d)) / 26
    """
    c = math.cos(math.pi / (N + 1))
    if kind == "5pt":
        return (1.0 - c, 1.0 + c)
    if kind == "7pt":
        return (1.0 - c, 1.0 + c)
    if kind == "27pt":
        ends = (1.0 + 2.0 * c, 1.0 - 2.0 * c)
        prods = [a * b * d for a in ends for b in ends for d in ends]
        return ((27.0 - max(prods)) / 26.0, (27.0 - min(prods)) / 26.0)
    raise ValueError(kind)


def start_vector(n: int, seed: int = SEED_LANCZOS) -> np.ndarray:
    """Start vector of the interval estimates: U[-1, 1] entries, unnormalised."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=n)


def lanczos_bounds(A: CSR, m: int = 20, seed: int = SEED_LANCZOS) -> tuple:
    """Extreme Ritz values of m-step Lanczos on D^{-1/2} A D^{-1/2}.

    Plain three-term Lanczos without reorthogonalisation from a U[-1,1] start
    vector; no safety margin is added.
    """
    from . import _native
    L = _native.lib()
    dh = np.ascontiguousarray(np.sqrt(jacobi_inverse(A)))
    w = np.empty(A.n)

    def scaled_matvec(v):
        L.inp_scaled_matvec(A.n, A.row_ptr.ctypes.data, A.col.ctypes.data,
                            A.val.ctypes.data, dh.ctypes.data, v.ctypes.data,
                            w.ctypes.data)
        return w.copy()

    v = start_vector(A.n, seed)
    v /= np.linalg.norm(v)
    v_prev = np.zeros_like(v)
    alphas, betas = [], []
    beta = 0.0
    for _ in range(min(m, A.n)):
        w = scaled_matvec(v)
        a = float(v @ w)
        w -= a * v + beta * v_prev
        alphas.append(a)
        beta = float(np.linalg.norm(w))
        if beta == 0.0:
            break
        betas.append(beta)
        v_prev, v = v, w / beta
    k = len(alphas)
    T = np.diag(alphas) + np.diag(betas[:k - 1], 1) + np.diag(betas[:k - 1], -1)
    ev = np.linalg.eigvalsh(T)
    return (float(ev[0]), float(ev[-1]))


def power_bounds(A: CSR, rtol: float = 1e-3, max_iter: int = 50,
                 seed: int = SEED_LANCZOS) -> tuple:
    """lambda_min = 0 and a power-method lambda_max of M^{-1}A, M = diag(A).

    Stops when successive estimates differ by less than rtol relative, or
    after max_iter steps (Sec. "The s-step PCG method with Chebyshev Krylov
    basis").
    """
    from . import _native
    L = _native.lib()
    dinv = jacobi_inverse(A)
    ones = np.ones(A.n)
    Av = np.empty(A.n)
    v = start_vector(A.n, seed)
    v /= np.linalg.norm(v)
    lam_old = 0.0
    lam = 0.0
    for _ in range(max_iter):
        L.inp_scaled_matvec(A.n, A.row_ptr.ctypes.data, A.col.ctypes.data, A.val.ctypes.data,
                            ones.ctypes.data, v.ctypes.data, Av.ctypes.data)
        w = dinv * Av
        lam = float(np.linalg.norm(w))
        v = w / lam
        if abs(lam - lam_old) < rtol * abs(lam):
            break
        lam_old = lam
    return (0.0, lam)


def workload(name: str, N: int | None = None) -> dict:
    """The standard synthetic workloads, by name.

    Returns a dict with the matrix, right-hand side and solver parameters.
    ``N`` overrides the grid size (for reduced test instances).
    """
    if name == "poisson5":          # 2D 5-point Poisson, closed-form interval
        N = N or 64
        A = poisson5(N)
        b = rhs_uniform(A.n)
        return dict(A=A, b=b, s=4, sweeps=2, interval=closed_form_bounds("5pt", N),
                    tol=1e-8)
    if name == "poisson7":          # 3D 7-point Poisson, Lanczos interval
        N = N or 128
        A = poisson7(N)
        b = rhs_uniform(A.n)
        return dict(A=A, b=b, s=4, sweeps=2, interval=lanczos_bounds(A), tol=1e-8)
    if name == "diffusion27":       # 27-point heterogeneous diffusion
        N = N or 192
        A = stencil("27pt", N, coeff_blocks(N))
        b = rhs_normal(A.n)
        return dict(A=A, b=b, s=6, sweeps=2, interval=lanczos_bounds(A), tol=1e-8)
    if name == "diffusion7":        # 7-point diffusion with k = exp(theta)
        N = N or 96
        theta = theta_field(N**3)
        A = stencil("7pt", N, np.exp(theta))
        b = rhs_uniform(A.n)
        return dict(A=A, b=b, s=4, sweeps=2, interval=lanczos_bounds(A), tol=1e-8,
                    theta=theta, x_target=x_target(A.n))
    if name == "hpcg27":            # the paper's per-GPU share: HPCG 27-point, b = 1
        N = N or 200
        A = hpcg27(N)
        return dict(A=A, b=np.ones(A.n), s=4, sweeps=30, interval=power_bounds(A), tol=1e-8)
    raise ValueError(f"unknown workload {name!r}")
