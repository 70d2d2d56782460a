"""Spectral helpers of the tests (scipy's ARPACK; no oracle code)."""
import scipy.sparse.linalg as spl

import sspcg_inputs as si


def kappa2(A) -> float:
    """kappa_2(A) = lambda_max / lambda_min of the SPD matrix A: with it,
    ||x - x*|| / ||x*|| <= kappa_2(A) ||b - A x|| / ||b|| bounds the error of
    any x by its residual."""
    S = si.to_scipy(A).tocsc()
    hi = spl.eigsh(S, k=1, which="LA", return_eigenvectors=False, tol=1e-8)[0]
    lo = spl.eigsh(S, k=1, sigma=0.0, which="LM", return_eigenvectors=False, tol=1e-8)[0]
    return float(hi / lo)
