"""Writes the oracle's gradient record of the differentiable form's workload.

7-point diffusion on 96^3 (kappa = exp(theta), theta ~ N(0, 0.5^2) per
cell), loss L = 0.5 ||x - x_target||^2 with x = A(theta)^{-1} b.  The
gradient follows the adjoint chain of the differentiable form: the forward
solve, the adjoint solve A lambda = x - x_target, the value gradient
-lambda_i x_j over the sparsity pattern, and its pull-back to theta through
the harmonic-mean assembly -- each step the oracle's own (``oracle.sspcg``,
``oracle.csr_value_grad``, ``oracle.diffusion7_theta_grad``), both solves by
Algorithm 1 (s = 4, two FGS sweeps, the workload's Lanczos interval) to a
relative residual of 1e-14.  The record holds the loss, ||dL/dtheta||, the
gradient at 16384 indices from ``sspcg_inputs.sample_indices``, its
projections on the 8 vectors of ``sspcg_inputs.probe_vectors``, and digests
of theta, b and x_target.  Only ``oracle`` and ``sspcg_inputs`` are used.

    python tests/golden/make_gradient_records.py
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import sspcg_inputs as si  # noqa: E402

OUT = os.path.join(HERE, "gradients")
TOL = 1e-14
N_SAMPLES = 16384
N_PROBES = 8


def make(N: int = 96) -> dict:
    w = si.workload("diffusion7", N=N)
    A, theta, b, xt = w["A"], w["theta"], w["b"], w["x_target"]
    interval = tuple(float(v) for v in w["interval"])
    t0 = time.time()
    x, rx = oracle.sspcg(A, b, s=w["s"], sweeps=w["sweeps"], interval=interval, tol=TOL,
                         max_outer=100000)
    lam, rl = oracle.sspcg(A, x - xt, s=w["s"], sweeps=w["sweeps"], interval=interval, tol=TOL,
                           max_outer=100000)
    g = oracle.diffusion7_theta_grad(A, theta, oracle.csr_value_grad(A, lam, x))
    seconds = time.time() - t0
    idx = si.sample_indices(A.n, N_SAMPLES)
    V = si.probe_vectors(A.n, N_PROBES)
    d = x - xt
    return dict(
        case=f"diffusion7_{N}_grad",
        what="oracle gradient of 0.5 ||x - x_target||^2 through two s-step solves",
        command="python tests/golden/make_gradient_records.py",
        workload="diffusion7", N=N, n=A.n, nnz=A.nnz, s=w["s"], sweeps=w["sweeps"],
        interval_hex=[interval[0].hex(), interval[1].hex()], tol=TOL,
        digest_theta=si.digest(theta), digest_b=si.digest(b), digest_x_target=si.digest(xt),
        forward_iters=int(rx["iters"]), adjoint_iters=int(rl["iters"]),
        status=[int(rx["status"]), int(rl["status"])],
        loss=float(0.5 * oracle.dot(d, d)),
        norm_g=float(np.sqrt(oracle.dot(g, g))),
        n_samples=int(idx.size), digest_indices=si.digest(idx),
        g_samples=[float(v) for v in g[idx]],
        n_probes=N_PROBES, projections=[float(oracle.dot(g, v)) for v in V],
        probe_norms=[float(np.sqrt(oracle.dot(v, v))) for v in V],
        oracle_seconds=round(seconds, 1), oracle_threads=oracle.threads(),
    )


def main() -> int:
    rec = make()
    os.makedirs(OUT, exist_ok=True)
    path = os.path.join(OUT, rec["case"] + ".json")
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    os.replace(path + ".tmp", path)
    print(f"{path}: forward {rec['forward_iters']}, adjoint {rec['adjoint_iters']} outer "
          f"iterations, {rec['oracle_seconds']} s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
