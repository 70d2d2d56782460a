"""Writes the oracle's solution records for the full-size workloads.

Each record summarises one CPU-oracle solve of a standard workload so that a
GPU test can check the device solution at the workload's real size without
running the oracle there (the 192^3 solve takes about half an hour on eight
host cores):

* the oracle's status, outer iterations and final relative residuals;
* ||x||_2;
* x at 2048 indices drawn with ``sspcg_inputs.sample_indices`` (16384 for
  the 192^3 workload, whose records also stand in for the full solution in
  the benchmark's error report);
* x^T v for the 8 vectors of ``sspcg_inputs.probe_vectors``;
* the Gram solve and basis: for the paper's own workload (HPCG 27-point
  200^3, b = 1, power-method interval) 30 FGS sweeps or the Cholesky solve;
  adaptive sweeps on the 192^3 system; the monomial basis on 128^3;
* the basis interval the solve used (exact, as float.hex), and digests of
  the matrix values and the right-hand side, so that a test can tell whether
  it rebuilt the same system.

The s-step records follow Algorithm 1 with Algorithm 2 and FGS Gram solves
(``oracle.sspcg``) run to a relative residual of 1e-14; the "pcg" records are
classical Jacobi PCG (``oracle.pcg``) to 1e-13 and serve as the reference
solution x_ref of the mixed-precision form.  Two solves that each reach a
relative residual tau can differ by up to kappa_2(A) tau; at tau = 1e-12 the
7-point 128^3 system (kappa_2 about 6.7e3) let the s-step solutions of two
correct implementations differ by 1.3e-10, so the s-step records go to 1e-14,
where such pairs agree to about 1e-13.  Only ``oracle`` and
``sspcg_inputs`` are used: no value here comes from the GPU library.

    python tests/golden/make_solution_records.py --list
    python tests/golden/make_solution_records.py --case diffusion27_192_s6_nu2
    python tests/golden/make_solution_records.py --all
"""
from __future__ import annotations

import argparse
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

OUT = os.path.join(HERE, "solutions")
N_SAMPLES = 2048
N_PROBES = 8
SSTEP_TOL = 1e-14
PCG_TOL = 1e-13


def _cases() -> dict:
    c = {}
    # 2D 5-point Poisson 64 x 64, closed-form interval, s = 4, nu = 2
    c["poisson5_64_s4_nu2"] = dict(workload="poisson5", N=64, method="sspcg", s=4, sweeps=2)
    c["poisson5_64_pcg"] = dict(workload="poisson5", N=64, method="pcg")
    # 3D 7-point Poisson 128^3, Lanczos interval, the s x nu grid
    for s in (2, 4, 6, 8):
        for nu in (1, 2, 3):
            if (s, nu) == (2, 1):       # does not converge (20 000 outer iterations)
                continue
            c[f"poisson7_128_s{s}_nu{nu}"] = dict(workload="poisson7", N=128, method="sspcg",
                                                  s=s, sweeps=nu)
    c["poisson7_128_pcg"] = dict(workload="poisson7", N=128, method="pcg")
    # 27-point heterogeneous diffusion 192^3, s = 6, nu = 2
    c["diffusion27_192_s6_nu2"] = dict(workload="diffusion27", N=192, method="sspcg", s=6,
                                       sweeps=2, samples=16384)
    c["diffusion27_192_pcg"] = dict(workload="diffusion27", N=192, method="pcg", samples=16384)
    # the paper's own workload (HPCG 27-point 200^3, b = 1, lambda_min = 0 and
    # power-method lambda_max): FGS with 30 sweeps and the Cholesky Gram solve
    c["hpcg27_200_s4_nu30"] = dict(workload="hpcg27", N=200, method="sspcg", s=4, sweeps=30)
    c["hpcg27_200_s6_cholesky"] = dict(workload="hpcg27", N=200, method="sspcg", s=6,
                                       sweeps=1, gram="cholesky")
    # adaptive sweeps on the benchmark system (stop sweeping once
    # ||m - W a|| <= 1e-3 ||m||, at most 30 sweeps) and the monomial basis
    # on the 7-point Poisson 128^3 system
    c["diffusion27_192_s6_adaptive"] = dict(workload="diffusion27", N=192, method="sspcg", s=6,
                                            sweeps=30, sweep_tol=1e-3)
    c["poisson7_128_s2_nu3_monomial"] = dict(workload="poisson7", N=128, method="sspcg", s=2,
                                             sweeps=3, basis="monomial")
    return c


CASES = _cases()


def record_path(case: str) -> str:
    return os.path.join(OUT, case + ".json")


def make(case: str) -> dict:
    spec = CASES[case]
    w = si.workload(spec["workload"], N=spec["N"])
    A, b = w["A"], w["b"]
    interval = tuple(float(v) for v in w["interval"])
    t0 = time.time()
    if spec["method"] == "sspcg":
        tol = SSTEP_TOL
        x, res = oracle.sspcg(A, b, s=spec["s"], sweeps=spec["sweeps"], interval=interval,
                              tol=tol, max_outer=100000, gram=spec.get("gram", "fgs"),
                              sweep_tol=spec.get("sweep_tol", 0.0),
                              basis=spec.get("basis", "chebyshev"))
    else:
        tol = PCG_TOL
        x, res = oracle.pcg(A, b, tol=tol, max_iter=200000)
    seconds = time.time() - t0
    idx = si.sample_indices(A.n, spec.get("samples", N_SAMPLES))
    V = si.probe_vectors(A.n, N_PROBES)
    rec = dict(
        case=case,
        what=(f"oracle s-step PCG (Algorithm 1, Chebyshev basis, "
              f"{'Cholesky' if spec.get('gram') == 'cholesky' else 'FGS'} Gram solves)"
              if spec["method"] == "sspcg" else "oracle classical Jacobi PCG"),
        command=f"python tests/golden/make_solution_records.py --case {case}",
        workload=spec["workload"], N=spec["N"], n=A.n, nnz=A.nnz, method=spec["method"],
        s=spec.get("s"), sweeps=spec.get("sweeps"), gram=spec.get("gram", "fgs"),
        sweep_tol=spec.get("sweep_tol", 0.0), basis=spec.get("basis", "chebyshev"),
        interval_hex=[interval[0].hex(), interval[1].hex()], interval=list(interval),
        tol=tol,
        digest_val=si.digest(A.val), digest_b=si.digest(b),
        status=int(res["status"]), iters=int(res["iters"]), relres=float(res["relres"]),
        relres_true=float(res["relres_true"]),
        norm_x=float(np.sqrt(oracle.dot(x, x))),
        n_samples=int(idx.size), digest_indices=si.digest(idx),
        x_samples=[float(v) for v in x[idx]],
        n_probes=N_PROBES, projections=[float(oracle.dot(x, v)) for v in V],
        probe_norms=[float(np.sqrt(oracle.dot(v, v))) for v in V],
        oracle_seconds=round(seconds, 1), oracle_threads=oracle.threads(),
    )
    return rec


def write(rec: dict) -> str:
    os.makedirs(OUT, exist_ok=True)
    path = record_path(rec["case"])
    with open(path + ".tmp", "w") as f:
        json.dump(rec, f, indent=0)
        f.write("\n")
    os.replace(path + ".tmp", path)
    return path


def load(case: str) -> dict:
    with open(record_path(case)) as f:
        return json.load(f)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--case", action="append", default=[])
    ap.add_argument("--all", action="store_true")
    ap.add_argument("--list", action="store_true")
    a = ap.parse_args(argv)
    if a.list:
        for c in CASES:
            print(c, "(written)" if os.path.exists(record_path(c)) else "")
        return 0
    todo = list(CASES) if a.all else a.case
    for c in todo:
        if c not in CASES:
            print(f"unknown case {c}", file=sys.stderr)
            return 2
    for c in todo:
        rec = make(c)
        path = write(rec)
        print(f"{c}: status {rec['status']}, {rec['iters']} iterations, relres "
              f"{rec['relres']:.3e} (true {rec['relres_true']:.3e}), "
              f"{rec['oracle_seconds']} s -> {os.path.relpath(path, ROOT)}", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
