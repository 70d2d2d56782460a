"""The committed oracle records are what the oracle and the input generators
produce today.

For every solution and gradient record of a system the host builds quickly
(up to 2.1 M rows), the generator must rebuild the recorded system (digests
of the values, right-hand side and sampling indices, the basis interval to
1e-10); the 2D Poisson 64^2
records are recomputed by the oracle in full and must match bit for bit, so
the records are reproducible from the oracle alone.
"""
import glob
import json
import os

import numpy as np
import pytest

import oracle
import sspcg_inputs as si

HERE = os.path.dirname(os.path.abspath(__file__))
SOLUTIONS = sorted(glob.glob(os.path.join(HERE, "golden", "solutions", "*.json")))
GRADIENTS = sorted(glob.glob(os.path.join(HERE, "golden", "gradients", "*.json")))
SMALL = 2_100_000


def _small(paths):
    out = []
    for p in paths:
        rec = json.load(open(p))
        if rec["n"] <= SMALL:
            out.append(p)
    return out


@pytest.mark.parametrize("path", _small(SOLUTIONS), ids=lambda p: os.path.basename(p)[:-5])
def test_solution_record_matches_generator(path):
    rec = json.load(open(path))
    w = si.workload(rec["workload"], N=rec["N"])
    assert si.digest(w["A"].val) == rec["digest_val"]
    assert si.digest(w["b"]) == rec["digest_b"]
    assert si.digest(si.sample_indices(rec["n"], rec["n_samples"])) == rec["digest_indices"]
    # the interval is an input the record carries exactly; the generator's
    # Lanczos estimate may differ from it in the last bits (its dot products
    # run in library code whose summation order depends on the host)
    rec_iv = [float.fromhex(h) for h in rec["interval_hex"]]
    assert np.allclose(w["interval"], rec_iv, rtol=1e-10, atol=0)
    assert rec["status"] == 0 and rec["relres"] <= rec["tol"]


@pytest.mark.parametrize("path", _small(GRADIENTS), ids=lambda p: os.path.basename(p)[:-5])
def test_gradient_record_matches_generator(path):
    rec = json.load(open(path))
    w = si.workload(rec["workload"], N=rec["N"])
    assert si.digest(w["theta"]) == rec["digest_theta"]
    assert si.digest(w["b"]) == rec["digest_b"]
    assert si.digest(w["x_target"]) == rec["digest_x_target"]
    rec_iv = [float.fromhex(h) for h in rec["interval_hex"]]
    assert np.allclose(w["interval"], rec_iv, rtol=1e-10, atol=0)
    assert rec["status"] == [0, 0]


@pytest.mark.parametrize("case", ["poisson5_64_s4_nu2", "poisson5_64_pcg"])
def test_small_records_are_reproduced_by_the_oracle(case):
    rec = json.load(open(os.path.join(HERE, "golden", "solutions", case + ".json")))
    w = si.workload(rec["workload"], N=rec["N"])
    interval = tuple(float.fromhex(h) for h in rec["interval_hex"])
    if rec["method"] == "sspcg":
        x, res = oracle.sspcg(w["A"], w["b"], s=rec["s"], sweeps=rec["sweeps"],
                              interval=interval, tol=rec["tol"], max_outer=100000)
    else:
        x, res = oracle.pcg(w["A"], w["b"], tol=rec["tol"], max_iter=200000)
    assert res["iters"] == rec["iters"]
    idx = si.sample_indices(rec["n"], rec["n_samples"])
    assert np.array_equal(x[idx], np.asarray(rec["x_samples"]))
    assert float(np.sqrt(oracle.dot(x, x))) == rec["norm_x"]
