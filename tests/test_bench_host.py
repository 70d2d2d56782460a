"""Host logic of bench.py (no GPU): the one-GPU guard, the byte models the
roofline divides by, and the guard on the counter-traffic record."""
import json
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_csr_model_matches_the_per_unit_figure():
    # 27-point 192^3: 12 B per nonzero, 4 B per row pointer, 8 B per vector
    # element read or written; one SpMV moves x and y
    n, nnz = 7077888, 189119224
    one = 12 * nnz + 4 * (n + 1) + 16 * n
    assert abs(one - 2.4105e9) < 1e6
    # the s launches of a matrix powers kernel add the epilogues: dinv read
    # and z_{q+1} written for q < s, z_{q-1} read for 2 <= q < s
    s = 6
    epi = 8 * n * (2 + 3 * (s - 2))
    assert bench.csr_family_bytes(n, nnz, s, 8) == s * one + epi


def test_stored_format_model():
    n, nnz, s = 1000, 26000, 4
    nval = bench.stored_values(n, nnz, True)
    assert nval == (nnz + n) // 2 and bench.stored_values(n, nnz, False) == nnz
    # uniform layout: no column indices; the half storage reads no dinv
    one = 8 * nval + 16 * n
    assert bench.spmv_bytes(n, nval, 8, 0.0) == one
    assert bench.spmv_bytes(n, nval, 8, 1.0) == one + 4 * nval
    with_dinv = bench.spmv_family_bytes(n, nval, s, 8, 0.0)
    without = bench.spmv_family_bytes(n, nval, s, 8, 0.0, dinv_read=False)
    assert with_dinv - without == 8 * n * (s - 1)
    assert without == s * one + 8 * n * (1 + 2 * (s - 2))


def test_phase_bytes_follow_the_solve_kernels():
    n, s = 100, 6
    pb = bench.phase_bytes(n, s, 8)
    assert pb["gram_update"] == (6 * s + 3) * 8 * n   # Z, Q, AZ, AQ, r, x in; Q, AQ, x out
    assert pb["gram_rect"] == 2 * s * 8 * n           # Q, AZ
    assert pb["xr"] == (s + 4) * 8 * n                # AQ, r, dinv in; r, z1 out


def test_traffic_record_is_ignored_when_the_code_changes(tmp_path, monkeypatch):
    src = tmp_path / "kernel.hip"
    src.write_text("// kernel v1\nint f() { return 1; }\n")
    rec = {"sources": [str(src)], "source_code_sha256": bench.code_digest([str(src)]),
           "traffic_bytes_per_launch": 123.0}
    path = tmp_path / "record.json"
    path.write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(path))
    assert bench.counter_traffic() == 123.0
    # comments and layout do not count
    src.write_text("// kernel v2, reworded\n/* a block\n comment */ int f()  {\n return 1; }\n")
    assert bench.counter_traffic() == 123.0
    src.write_text("// kernel v2\nint f() { return 2; }\n")
    assert bench.counter_traffic() is None
    path.write_text("not json")
    assert bench.counter_traffic() is None


def test_roofline_bytes_per_launch_at_192():
    # stored format of the 27-point 192^3 matrix: the diagonal and 13 upper
    # offsets per row (8 B each), x read and y written, the epilogues' z
    # vectors; averaged over the s = 6 launches of one matrix powers kernel
    n, nnz, s = 7077888, 189119224, 6
    nval = bench.stored_values(n, nnz, True)
    per_launch = bench.spmv_family_bytes(n, nval, s, 8, 0.0, dinv_read=False) / s
    assert per_launch == 982969312.0


def test_error_vs_record_estimates_the_relative_error():
    import numpy as np
    import torch
    import sspcg_inputs as si
    n, k = 200000, 4096
    rng = np.random.default_rng(7)
    xo = rng.normal(size=n)
    delta = 1e-9 * rng.normal(size=n)
    idx = si.sample_indices(n, k)
    rec = {"n": n, "n_samples": k, "x_samples": xo[idx].tolist(),
           "norm_x": float(np.linalg.norm(xo)), "what": "test", "tol": 0.0, "iters": 0,
           "case": "synthetic"}
    e = bench.error_vs_record(torch.from_numpy(xo + delta), rec)
    true = np.linalg.norm(delta) / np.linalg.norm(xo)
    assert abs(e["rel_error_sampled"] / true - 1) < 0.1
    assert e["max_sampled_diff_rel"] <= np.abs(delta).max() / np.abs(xo[idx]).max() * 1.0001
    e0 = bench.error_vs_record(torch.from_numpy(xo), rec)
    assert e0["rel_error_sampled"] == 0.0 and e0["max_sampled_diff_rel"] == 0.0


def test_oracle_record_rejects_other_inputs():
    import numpy as np
    import sspcg_inputs as si
    A = si.poisson5(64)
    b = si.rhs_uniform(A.n)
    rec = bench.oracle_record("poisson5_64_s4_nu2", A, b)
    assert rec is not None and rec["n"] == A.n
    assert bench.oracle_record("poisson5_64_s4_nu2", A, b + 1.0) is None
    assert bench.oracle_record("no_such_case", A, b) is None


def _fake_rocpd(path, kernels, counters):
    import sqlite3
    con = sqlite3.connect(path)
    con.execute("create table kernels (name text, duration integer)")
    con.execute("create table counters_collection (dispatch_id integer, kernel_name text, "
                "counter_name text, value real)")
    con.executemany("insert into kernels values (?, ?)", kernels)
    con.executemany("insert into counters_collection values (?, ?, ?, ?)", counters)
    con.commit()
    con.close()


def test_counter_passes_make_the_traffic_record(tmp_path, monkeypatch):
    spmv = "void sspcg::(anonymous namespace)::k_spmv<double, {}>(sspcg::Sell<double>, double const*)"
    f, w = tmp_path / "f", tmp_path / "w"
    f.mkdir()
    w.mkdir()
    # the 1 GiB copy (FETCH_SIZE counts half its reads) and a smaller copy
    fetch = [(1, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 524288.0),
             (2, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 1.0)]
    write = [(1, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 1048576.0),
             (2, "__amd_rocclr_copyBuffer", "WRITE_SIZE", 2.0)]
    for m, kib in ((0, 1000.0), (1, 2000.0), (2, 3000.0)):
        fetch += [(10 + m, spmv.format(m), "FETCH_SIZE", kib), (20 + m, spmv.format(m), "FETCH_SIZE", kib)]
        write += [(10 + m, spmv.format(m), "WRITE_SIZE", 100.0), (20 + m, spmv.format(m), "WRITE_SIZE", 100.0)]
    _fake_rocpd(f / "kern_results.db", [], fetch)
    _fake_rocpd(w / "kern_results.db", [], write)
    monkeypatch.setattr(bench, "TRAFFIC_RECORD", str(tmp_path / "rec.json"))
    rec = bench.traffic_record(str(f), str(w), 6)
    assert rec["calibration"]["fetch_scale"] == 2.0 and rec["calibration"]["write_scale"] == 1.0
    per = {m: (2 * kib + 100.0) * 1024 for m, kib in ((0, 1000.0), (1, 2000.0), (2, 3000.0))}
    assert rec["modes"]["k_spmv<double, 1>"]["traffic_bytes"] == per[1]
    assert abs(rec["traffic_bytes_per_launch"] - (per[1] + 4 * per[2] + per[0]) / 6) < 1e-6
    # the record guards itself against source changes
    assert bench.counter_traffic() == rec["traffic_bytes_per_launch"]


def test_trace_summary_table(tmp_path):
    k0 = "void sspcg::(anonymous namespace)::k_spmv<double, 0>(sspcg::Sell<double>)"
    _fake_rocpd(tmp_path / "b_results.db", [(k0, 200000), (k0, 220000), ("k_norm_step(x)", 5000)], [])
    t = bench.trace_summary(str(tmp_path))
    assert "| `k_spmv<double, 0>` | 2 | 0.42 | 210.0 | 200.0 | 220.0 |" in t
    assert "`k_norm_step`" in t
