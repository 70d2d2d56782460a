"""FP64 solution parity with the oracle at the workloads' real sizes.

1. Against the oracle's committed solution records (written by
   tests/golden/make_solution_records.py from the CPU oracle alone): the
   2D Poisson 64^2 system, the 7-point Poisson 128^3 (s, nu) grid, the
   27-point heterogeneous 192^3 benchmark system (also with adaptive
   sweeps), the 7-point 128^3 system in the monomial basis, and the paper's
   own workload (HPCG 27-point 200^3, b = 1) with 30 FGS sweeps and with the
   Cholesky Gram solve.  Both sides run
   Algorithm 1 with the same interval, s and nu to the record's relative
   residual (1e-14; classical PCG 1e-13): two correct solves to tau differ by
   up to kappa_2(A) tau, so 1e-12 would not support the 1e-10 bar on the
   128^3 system.  The device solution must agree with the oracle's to 1e-10 in the
   sampled entries, the norm and the projections on seeded random vectors,
   and in the 2-norm error estimated from the uniformly sampled entries.
2. At the benchmark tolerance 1e-8, where the two iterations may part by
   rounding: both solutions lie within the forward-error bound
   kappa_2(A) ||b - A x|| / ||b|| of x_ref (oracle PCG to 1e-13), and the
   device's outer-iteration count lies within the spread of the oracle's runs
   whose Gram entries are moved by one unit in the last place (tests/spread.py:
   within four standard deviations of 24 such runs; five runs, as first
   planned, sample too little of a distribution that spans 291..483 on the
   64^2 system).
3. The mixed form at 192^3, refined to a true residual of 1e-12, against the
   oracle's PCG record: the same 1e-10 bar as the FP64 solver.
4. The differentiable form at its workload's size (7-point diffusion 96^3):
   the gradient through the device's forward and adjoint solves against the
   oracle's gradient record (tests/golden/make_gradient_records.py), 1e-10.
"""
import glob
import json
import os

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
HERE = os.path.dirname(os.path.abspath(__file__))
RECORDS = sorted(glob.glob(os.path.join(HERE, "golden", "solutions", "*.json")))
GRADIENTS = sorted(glob.glob(os.path.join(HERE, "golden", "gradients", "*.json")))
SOLUTION_TOL = 1e-10


def load_system(rec):
    w = si.workload(rec["workload"], N=rec["N"])
    A, b = w["A"], w["b"]
    assert si.digest(A.val) == rec["digest_val"] and si.digest(b) == rec["digest_b"], \
        "the input generator no longer builds the recorded system"
    interval = (float.fromhex(rec["interval_hex"][0]), float.fromhex(rec["interval_hex"][1]))
    return A, b, interval


def against_record(x, rec, idx):
    """Relative differences of a device solution from an oracle record: the
    2-norm error estimated from the sampled entries, the largest sampled
    difference, the norm, and the largest projection on the seeded probes."""
    xs = x[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    xo = np.asarray(rec["x_samples"])
    nx = torch.linalg.vector_norm(x).item()
    d = xs - xo
    est = np.sqrt(rec["n"] / idx.size * np.sum(d * d)) / rec["norm_x"]
    worst = np.abs(d).max() / np.abs(xo).max()
    xh = x.cpu().numpy()
    V = si.probe_vectors(rec["n"], rec["n_probes"])
    proj = np.array([oracle.dot(xh, v) for v in V])
    del V
    pe = np.abs(proj - np.asarray(rec["projections"])) \
        / (rec["norm_x"] * np.asarray(rec["probe_norms"]))
    return est, worst, abs(nx - rec["norm_x"]) / rec["norm_x"], pe.max()


@pytest.mark.parametrize("path", RECORDS, ids=[os.path.basename(p)[:-5] for p in RECORDS])
def test_solution_matches_oracle_record(path):
    rec = json.load(open(path))
    print(f"[record] {rec['case']}: n={rec['n']} method={rec['method']} tol={rec['tol']}",
          flush=True)
    A, b, interval = load_system(rec)
    M = P.Matrix.from_csr(A, device=DEV)
    bd = torch.from_numpy(b).to(DEV)
    if rec["method"] == "sspcg":
        x, info = P.solve(M, bd, s=rec["s"], sweeps=rec["sweeps"], interval=interval,
                          tol=rec["tol"], max_outer=100000, gram=rec.get("gram", "fgs"),
                          sweep_tol=rec.get("sweep_tol", 0.0),
                          basis=rec.get("basis", "chebyshev"))
    else:
        x, info = P.pcg(M, bd, tol=rec["tol"], max_iter=200000)
    assert info["status"] == P.OK and rec["status"] == 0
    assert info["relres"] <= rec["tol"]
    idx = si.sample_indices(rec["n"], rec["n_samples"])
    assert si.digest(idx) == rec["digest_indices"]
    est, worst, nd, pe = against_record(x, rec, idx)
    print(f"[record] {rec['case']}: device {info['outer_iters']} iterations, oracle "
          f"{rec['iters']}; sampled 2-norm error {est:.2e}, worst sample {worst:.2e}, "
          f"norm {nd:.2e}, projections {pe:.2e}")
    assert est <= SOLUTION_TOL
    assert worst <= SOLUTION_TOL
    assert nd <= SOLUTION_TOL
    assert pe <= SOLUTION_TOL
    # The iteration counts are reported, not compared: with one or two FGS
    # sweeps they are set by rounding (60 perturbed oracle runs of the 64^2
    # system spread over +-20 % of their mean at 1e-12, tests/spread.py, where
    # the device count is checked against that spread; s = 2, nu = 2 on 128^3
    # took 27057 outer iterations in the oracle and 14713 on the device, with
    # the same solution).


@pytest.mark.parametrize("name,N", [("poisson5", 64), ("diffusion27", 24)])
def test_tau_1e8_forward_error_and_iteration_spread(name, N):
    print(f"[tau 1e-8] {name} N={N}", flush=True)
    w = si.workload(name, N=N)
    A, b = w["A"], w["b"]
    s, nu, tol = w["s"], w["sweeps"], 1e-8
    x_ref, rr = oracle.pcg(A, b, tol=1e-13)
    assert rr["status"] == oracle.OK
    kap = kappa2(A)
    M = P.Matrix.from_csr(A, device=DEV)
    x, info = P.solve(M, torch.from_numpy(b).to(DEV), s=s, sweeps=nu, interval=w["interval"],
                      tol=tol)
    assert info["status"] == P.OK
    xg = x.cpu().numpy()
    S = si.to_scipy(A)
    nb, nr = np.linalg.norm(b), np.linalg.norm(x_ref)

    def fwd(v):
        err = np.linalg.norm(v - x_ref) / nr
        bound = kap * np.linalg.norm(b - S @ v) / nb
        return err, bound

    eg, bg = fwd(xg)
    for seed in range(6):      # 0: unperturbed; 1..5: one-ulp Gram perturbations
        xo, ro = oracle.sspcg(A, b, s=s, sweeps=nu, interval=w["interval"], tol=tol,
                              perturb_seed=seed)
        assert ro["status"] == oracle.OK
        eo, bo = fwd(xo)
        assert eo <= bo
        if seed == 0:
            diff = np.linalg.norm(xg - xo) / np.linalg.norm(xo)
    counts = perturbed_counts(A, b, s=s, sweeps=nu, interval=w["interval"], tol=tol, runs=24)
    print(f"[tau 1e-8] {name} {N}: kappa_2 {kap:.3e}; device {info['outer_iters']} outer, "
          f"error vs x_ref {eg:.2e} (bound {bg:.2e}); oracle counts {counts.min()}.."
          f"{counts.max()} (mean {counts.mean():.1f}, sd {counts.std():.1f}); "
          f"device vs unperturbed oracle {diff:.2e}")
    assert eg <= bg
    assert within_spread(info["outer_iters"], counts)


def test_mixed_refinement_reaches_1e10_against_oracle_record():
    """The mixed form (FP32 inner s-step solves inside FP64 iterative
    refinement) on the 27-point 192^3 benchmark system, refined to a true
    relative residual of 1e-12: its solution agrees with the oracle's
    classical PCG record (relative residual 1e-13) to 1e-10, the accuracy the
    FP64 solver is held to.  (At a residual of 1e-10 the error is about
    1e-10 for both the mixed and the FP64 solve: a residual bounds the error
    only up to kappa_2(A).)"""
    path = os.path.join(HERE, "golden", "solutions", "diffusion27_192_pcg.json")
    rec = json.load(open(path))
    print(f"[mixed record] {rec['case']}: n={rec['n']}", flush=True)
    w = si.workload("diffusion27", N=192)
    A, b = w["A"], w["b"]
    assert si.digest(A.val) == rec["digest_val"] and si.digest(b) == rec["digest_b"]
    M = P.Matrix.from_csr(A, fp32=True, device=DEV)
    x, info = P.solve(M, torch.from_numpy(b).to(DEV), s=w["s"], sweeps=w["sweeps"],
                      interval=w["interval"], tol=1e-12, precision="mixed")
    assert info["status"] == P.OK and info["relres"] <= 1e-12
    idx = si.sample_indices(rec["n"], rec["n_samples"])
    est, worst, nd, pe = against_record(x, rec, idx)
    print(f"[mixed record] {info['refinements']} refinements, {info['outer_iters']} inner "
          f"iterations; sampled 2-norm error {est:.2e}, worst sample {worst:.2e}, "
          f"norm {nd:.2e}, projections {pe:.2e}")
    assert max(est, worst, nd, pe) <= SOLUTION_TOL


@pytest.mark.parametrize("path", GRADIENTS, ids=[os.path.basename(p)[:-5] for p in GRADIENTS])
def test_gradient_matches_oracle_record(path):
    """dL/dtheta of L = 0.5 ||x - x_target||^2, x = A(theta)^{-1} b, through
    the device's forward and adjoint s-step solves (both to the record's
    1e-14) and its gradient kernels, against the oracle's: the loss, the
    sampled entries, the norm and the projections agree to 1e-10."""
    rec = json.load(open(path))
    print(f"[gradient record] {rec['case']}: n={rec['n']}", flush=True)
    w = si.workload(rec["workload"], N=rec["N"])
    A, theta, b, xt = w["A"], w["theta"], w["b"], w["x_target"]
    assert (si.digest(theta), si.digest(b), si.digest(xt)) == \
        (rec["digest_theta"], rec["digest_b"], rec["digest_x_target"])
    interval = (float.fromhex(rec["interval_hex"][0]), float.fromhex(rec["interval_hex"][1]))
    M = P.Matrix.from_csr(A, device=DEV)
    opts = dict(s=rec["s"], sweeps=rec["sweeps"], interval=interval, tol=rec["tol"])
    th = torch.from_numpy(theta).to(DEV).requires_grad_(True)
    x = P.DiffusionSolve.apply(th, torch.from_numpy(b).to(DEV), M, opts)
    loss = 0.5 * torch.sum((x - torch.from_numpy(xt).to(DEV)) ** 2)
    loss.backward()
    g = th.grad.detach()
    idx = si.sample_indices(rec["n"], rec["n_samples"])
    assert si.digest(idx) == rec["digest_indices"]
    gs = g[torch.from_numpy(idx).to(DEV)].cpu().numpy()
    go = np.asarray(rec["g_samples"])
    d = gs - go
    est = np.sqrt(rec["n"] / idx.size * np.sum(d * d)) / rec["norm_g"]
    worst = np.abs(d).max() / np.abs(go).max()
    ng = torch.linalg.vector_norm(g).item()
    gh = g.cpu().numpy()
    V = si.probe_vectors(rec["n"], rec["n_probes"])
    pe = max(abs(oracle.dot(gh, v) - p) / (rec["norm_g"] * pn)
             for v, p, pn in zip(V, rec["projections"], rec["probe_norms"]))
    del V
    le = abs(loss.item() - rec["loss"]) / rec["loss"]
    print(f"[gradient record] loss {le:.2e}, sampled 2-norm error {est:.2e}, worst sample "
          f"{worst:.2e}, norm {abs(ng - rec['norm_g']) / rec['norm_g']:.2e}, projections {pe:.2e}")
    assert max(le, est, worst, abs(ng - rec["norm_g"]) / rec["norm_g"], pe) <= SOLUTION_TOL
