"""Step-by-step run of the oracle's s-step PCG that keeps every state.

Composes the oracle's primitives in the order of Algorithm 1 (outer
iteration) and Algorithm 2 (matrix powers kernel), recording the state at
the start of each outer iteration.  Used by the pin tests (invariants that
need intermediate states) and by the GPU teacher-forcing tests.
"""
from __future__ import annotations

import numpy as np

import oracle


def trace(A, b, *, s, sweeps, interval, tol, max_outer, x0=None, gram="fgs", sweep_tol=0.0):
    """Returns (x, status, states).

    states[k] is a dict holding, at the start of outer iteration k (before
    W_k is formed): x, r, Z, P (the MPK output used to form Q_k), Q, AQ, and,
    once computed, W, b1, alpha, and for the beta system B2, beta, and the
    MPK output of r^{(k+1)} (Znext, Pnext).
    """
    dinv = oracle.jacobi_inverse(A)
    x = np.zeros(A.n) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - oracle.spmv(A, x)
    nb = np.sqrt(oracle.dot(b, b))
    Z, P = oracle.mpk(A, dinv, r, s, interval)
    Q, AQ = Z.copy(), P[1:].copy()
    states = []
    solve = (lambda W, B: oracle.chol_solve(W, B)) if gram == "cholesky" else \
        (lambda W, B: oracle.fgs(W, B, sweeps, sweep_tol))
    status = oracle.NOT_CONVERGED
    for k in range(max_outer):
        st = dict(k=k, x=x.copy(), r=r.copy(), Z=Z.copy(), P=P.copy(), Q=Q.copy(), AQ=AQ.copy())
        states.append(st)
        W, b1 = oracle.gram(Q, AQ, P[0])
        al, code = solve(W, b1)
        st.update(W=W, b1=b1, alpha=al)
        if code != oracle.OK:
            status = code
            break
        oracle.xr_update(Q, AQ, al, x, r)
        relres = np.sqrt(oracle.dot(r, r)) / nb
        st["relres"] = relres
        if relres <= tol:
            status = oracle.OK
            break
        Z, P = oracle.mpk(A, dinv, r, s, interval)
        B2 = oracle.gram_rect(Q, P[1:])
        be, code = solve(W, B2)
        st.update(B2=B2, beta=be, Znext=Z.copy(), Pnext=P.copy())
        if code != oracle.OK:
            status = code
            break
        oracle.block_update(Z, Q, P[1:], AQ, be)
    return x, status, states
