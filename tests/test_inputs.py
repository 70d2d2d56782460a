"""Pins of the seeded input generators (matrices, coefficients, intervals)."""
import numpy as np
import pytest
import scipy.sparse as sp

import sspcg_inputs as si


@pytest.mark.parametrize("kind,N", [("5pt", 3), ("5pt", 17), ("7pt", 3), ("7pt", 9),
                                    ("27pt", 3), ("27pt", 8)])
def test_nnz_formula(kind, N):
    A = si.stencil(kind, N)
    assert A.nnz == si.nnz_formula(kind, N)
    assert A.row_ptr[-1] == A.nnz


@pytest.mark.parametrize("kind,N", [("5pt", 13), ("7pt", 7), ("27pt", 6)])
def test_symmetric_sorted_and_constant_reduction(kind, N):
    n = N * N if kind == "5pt" else N**3
    kap = np.exp(np.random.default_rng(7).normal(0, 1, n))
    A = si.stencil(kind, N, kap)
    S = si.to_scipy(A)
    assert abs(S - S.T).max() == 0.0
    for i in range(A.n):
        c = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        assert np.all(np.diff(c) > 0) and i in c
    # k == 1 reproduces the constant-coefficient stencil exactly
    A1 = si.stencil(kind, N, np.ones(n))
    A0 = si.stencil(kind, N)
    assert np.array_equal(A1.val, A0.val) and np.array_equal(A1.col, A0.col)
    deg = {"5pt": 4, "7pt": 6, "27pt": 26}[kind]
    D = si.to_scipy(A0).diagonal()
    assert np.all(D == deg)
    off = A0.val[A0.col != np.repeat(np.arange(A0.n), np.diff(A0.row_ptr))]
    assert np.all(off == -1.0)


@pytest.mark.parametrize("kind,N,kap", [("27pt", 16, "blocks"), ("7pt", 9, "theta"),
                                        ("5pt", 11, None)])
def test_c_assembler_matches_numpy_definition(kind, N, kap):
    n = N * N if kind == "5pt" else N**3
    kv = si.coeff_blocks(N) if kap == "blocks" else (np.exp(si.theta_field(n)) if kap else None)
    A = si.stencil(kind, N, kv)
    B = si.stencil_numpy(kind, N, kv)
    assert np.array_equal(A.row_ptr, B.row_ptr)
    assert np.array_equal(A.col, B.col)
    assert np.array_equal(A.val, B.val)


def test_diffusion_row_sums_vanish_in_interior():
    """Interior rows of the diffusion operator annihilate constants."""
    N = 8
    kap = si.coeff_blocks(N, block=4)
    A = si.stencil("27pt", N, kap)
    y = si.to_scipy(A) @ np.ones(A.n)
    z, yy, x = np.unravel_index(np.arange(A.n), (N, N, N))
    interior = (x > 0) & (x < N - 1) & (yy > 0) & (yy < N - 1) & (z > 0) & (z < N - 1)
    assert np.abs(y[interior]).max() < 1e-12 * np.abs(A.val).max()


@pytest.mark.parametrize("kind,N", [("5pt", 12), ("7pt", 6), ("27pt", 5), ("27pt", 6)])
def test_closed_form_eigenvalues(kind, N):
    """Closed-form extreme eigenvalues of D^{-1}A against a dense eigensolver."""
    A = si.stencil(kind, N)
    M = si.to_scipy(A).toarray()
    d = np.diag(M)
    ev = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    lo, hi = si.closed_form_bounds(kind, N)
    assert abs(lo - ev[0]) < 1e-12
    assert abs(hi - ev[-1]) < 1e-12


def test_closed_form_values_of_standard_workloads():
    lo, hi = si.closed_form_bounds("5pt", 64)
    assert abs(lo - 1.1677732e-3) < 1e-10 and abs(hi - 1.9988322) < 1e-7


def test_lanczos_and_power_bounds_lie_inside_spectrum():
    A = si.stencil("7pt", 8, np.exp(si.theta_field(512)))
    M = si.to_scipy(A).toarray()
    d = np.diag(M)
    ev = np.linalg.eigvalsh(M / np.sqrt(np.outer(d, d)))
    lo, hi = si.lanczos_bounds(A)
    # Ritz values interlace: inside [lambda_min, lambda_max]
    assert ev[0] - 1e-12 <= lo <= hi <= ev[-1] + 1e-12
    assert hi > 0.99 * ev[-1]
    plo, phi = si.power_bounds(A)
    assert plo == 0.0 and phi <= ev[-1] + 1e-12 and phi > 0.9 * ev[-1]


def test_seeded_generators_reproducible():
    assert np.array_equal(si.rhs_normal(100), si.rhs_normal(100))
    assert not np.array_equal(si.rhs_normal(100), si.rhs_uniform(100))
    k = si.coeff_blocks(16)
    assert k.min() >= 1e-2 and k.max() <= 1e2
    assert len(np.unique(k)) == 8
    u = si.unit_direction(50)
    assert abs(np.linalg.norm(u) - 1) < 1e-15
