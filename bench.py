"""Time-to-tolerance benchmark of the s-step PCG hot path on one MI355X.

Workload: 3D 27-point variable-coefficient diffusion on a 192^3 grid
(n = 7,077,888, nnz = 189,119,224), coefficients log-uniform over
[1e-2, 1e2] on 8^3 blocks, b ~ N(0,1), Jacobi preconditioner, s = 6, two FGS
sweeps, Chebyshev interval from 20-step Lanczos, tolerance 1e-8.  All inputs
are seeded and synthetic.

One step = one FP64 s-step PCG solve to tolerance plus one mixed-precision
(FP32 inner, FP64 refinement) solve to the same tolerance, inputs resident in
HBM.  `value` is the FP64 time to tolerance (median over the timed steps).
The roofline object covers the matrix powers kernel (the SpMV launches with
the fused Chebyshev/Jacobi epilogue), timed by HIP events around that phase
of every outer iteration inside the timed solves.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "time to rel-res 1e-8 (FP64 vs mixed) + HBM GB/s, 27-pt 192^3, 1 GPU"


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def stored_values(n: int, nnz: int, symmetric: bool) -> int:
    """Matrix values one SpMV has to stream: every nonzero, or with the
    symmetric half storage the diagonal and one triangle."""
    return (nnz + n) // 2 if symmetric else nnz


def spmv_bytes(n: int, nval: int, elem: int, col_frac: float) -> float:
    """Algorithmic bytes of one SpMV: the nval matrix values (elem each), the
    column indices of the entries stored with explicit columns (4 bytes,
    col_frac of them; slices with a shared offset list store none), the input
    vector read once and the output written once (2 n elem).  The zero
    padding of the sliced layout is not counted."""
    return elem * nval + 4 * col_frac * nval + 2 * n * elem


def spmv_family_bytes(n: int, nval: int, s: int, elem: int, col_frac: float = 1.0,
                      dinv_read: bool = True) -> float:
    """Algorithmic bytes of one matrix powers kernel (s SpMV launches): s
    SpMVs plus the epilogues, z_{q+1} written and (dinv_read) dinv read for
    q < s, and z_{q-1} read for 2 <= q < s (n elem each).  The symmetric half
    storage streams each row's diagonal with its values, so its epilogue
    forms 1/a_ii there instead of reading dinv."""
    per = 2 if dinv_read else 1
    epi = sum((per if q == 1 else per + 1) * n * elem for q in range(1, s))
    return s * spmv_bytes(n, nval, elem, col_frac) + epi


def csr_family_bytes(n: int, nnz: int, s: int, elem: int) -> float:
    """The same with a plain CSR stream: 4-byte column index per nonzero and
    a 4-byte row pointer per row."""
    return spmv_family_bytes(n, nnz, s, elem, 1.0) + s * 4 * (n + 1)


def phase_bytes(n: int, s: int, elem: int) -> dict:
    """Algorithmic bytes of the other phases per launch, as the solve runs
    them: its block update also applies the previous x += Q alpha (x read
    and written), so its x/r update touches neither x nor Q."""
    return {
        "gram_update": (6 * s + 3) * n * elem,   # read Z, Q, AZ, AQ, r, x; write Q, AQ, x
        "gram_rect": 2 * s * n * elem,           # read Q, AZ
        "xr": (s + 4) * n * elem,                # read AQ, r, dinv; write r, z1
    }


def build_workload(N: int):
    import sspcg_inputs as si
    t0 = time.time()
    A = si.stencil("27pt", N, si.coeff_blocks(N))
    b = si.rhs_normal(A.n)
    t1 = time.time()
    interval = si.lanczos_bounds(A)
    log(f"[bench] workload 27pt {N}^3: n={A.n} nnz={A.nnz} assembly {t1 - t0:.1f}s, "
        f"lanczos {time.time() - t1:.1f}s, interval {interval}")
    return A, b, interval


def si_start_vector(n: int):
    import sspcg_inputs as si
    return si.start_vector(n)


def host_description() -> dict:
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model}


def cpu_baseline(A, b, interval, s, sweeps, outer_iters_gpu, sample_outer, bytes_per_outer):
    """The oracle on the host, on a bounded sample of the same solve.

    Two runs of the oracle's FP64 s-step solve, of 2 and 2 + sample_outer
    outer iterations; their difference times sample_outer outer iterations
    with the setup (diagonal, r0, first basis) taken out.  Scaled by the
    GPU's outer-iteration count to tolerance."""
    import oracle
    oracle.build()
    times = []
    for k in (2, 2 + sample_outer):
        t0 = time.time()
        _, res = oracle.sspcg(A, b, s=s, sweeps=sweeps, interval=interval, tol=1e-30,
                              max_outer=k)
        times.append(time.time() - t0)
        assert res["iters"] == k
    per_outer = (times[1] - times[0]) / sample_outer
    return {
        "value": per_outer * outer_iters_gpu, "unit": "s", "cores": oracle.threads(),
        "kind": "oracle",
        "sample": (f"{sample_outer} outer iterations of the FP64 s-step solve on the same "
                   f"system, timed as the difference of a {2 + sample_outer}- and a "
                   f"2-iteration run ({times[1]:.1f} s and {times[0]:.1f} s wall; setup "
                   f"excluded), scaled by the GPU's {outer_iters_gpu} outer iterations to "
                   "tolerance"),
        "seconds_per_outer": per_outer,
        "gbs": bytes_per_outer / per_outer / 1e9,
        "gbs_bytes_model": "CSR stream and the fused-pass vector traffic per outer iteration",
        **host_description(),
    }


TRIAD_N = 1 << 27       # 1 GiB per operand: far past the 256 MB Infinity Cache


def triad_peak(P, torch, dev, reps=10):
    """Achievable HBM rate: the library's STREAM triad over three 1 GiB
    arrays, best of `reps` launches (HIP events on the current stream)."""
    a = torch.empty(TRIAD_N, dtype=torch.float64, device=dev)
    b = torch.ones_like(a)
    c = torch.ones_like(a)
    P.stream_triad(a, b, c, 0.5)
    best = float("inf")
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        P.stream_triad(a, b, c, 0.5)
        e1.record()
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / 1e3)
    nbytes = 3 * 8 * TRIAD_N
    ok = bool(torch.all(a == 1.5).item())
    del a, b, c
    if not ok:
        raise RuntimeError("stream triad produced wrong values")
    return {"gbs": nbytes / best / 1e9, "bytes": nbytes, "seconds": best}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--N", type=int, default=192)
    ap.add_argument("--s", type=int, default=6)
    ap.add_argument("--sweeps", type=int, default=2)
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-outer", type=int, default=20)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-profile", action="store_true",
                    help="time without the per-phase HIP events")
    ap.add_argument("--mode", choices=["solve", "kernels", "paper", "configs", "seeds",
                                       "traffic-record", "trace-summary", "units-summary"],
                    default="solve",
                    help="kernels: a few launches of each hot kernel on the workload and a "
                         "copy kernel of known size (for rocprofv3 counter passes); paper: the "
                         "paper's Gram-solve experiments on its own workload shape; seeds: the "
                         "FP64 and mixed solves for several right-hand sides")
    ap.add_argument("--paper-N", type=int, default=200)
    ap.add_argument("--paper-out", default=None,
                    help="paper mode: also write the per-iteration histories to this JSON file")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--trace-dir", default="gpurun_out/prof_bench",
                    help="trace-summary: output directory of a rocprofv3 --kernel-trace run")
    ap.add_argument("--units-dirs", nargs=2, default=["gpurun_out/pmc_k1", "gpurun_out/pmc_k2"],
                    help="units-summary: output directories of the two unit-counter passes")
    ap.add_argument("--fetch-dir", default="gpurun_out/pmc_FETCH_SIZE",
                    help="traffic-record: output directory of the rocprofv3 --pmc FETCH_SIZE pass")
    ap.add_argument("--write-dir", default="gpurun_out/pmc_WRITE_SIZE",
                    help="traffic-record: output directory of the rocprofv3 --pmc WRITE_SIZE pass")
    args = ap.parse_args()
    if args.mode == "trace-summary":
        print(trace_summary(args.trace_dir))
        return 0
    if args.mode == "units-summary":
        print(units_summary(args.units_dirs[0], args.units_dirs[1]))
        return 0
    if args.mode == "traffic-record":
        # host only: turns two counter passes over --mode kernels into the
        # traffic record the roofline object reads
        rec = traffic_record(args.fetch_dir, args.write_dir, args.s)
        print(json.dumps(rec, indent=1))
        return 0

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus} GPUs, WORLD_SIZE={world}): "
              "this build measures the single-GPU hot path; multi-GPU sharding is not built.",
              file=sys.stderr)
        return 2

    import torch
    import paper_2603_09790_amd as P

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.mode == "configs":
        print(json.dumps(other_configs(P, torch, dev, args)), flush=True)
        return 0
    if args.mode == "seeds":
        print(json.dumps(seed_spread(P, torch, dev, args)), flush=True)
        return 0
    if args.mode == "paper":
        out = paper_experiments(P, torch, dev, args)
        print(json.dumps(out["summary"]), flush=True)
        if args.paper_out:
            json.dump(out, open(args.paper_out, "w"))
        return 0

    A, b_np, interval = build_workload(args.N)
    t0 = time.time()
    M = P.Matrix.from_csr(A, fp32=not args.no_mixed, device=dev)
    info_m = M.info()
    col_frac = 1.0 - info_m["shared_slices"] / info_m["slices"]
    sym = bool(info_m["symmetric"])
    nval = stored_values(A.n, A.nnz, sym)
    log(f"[bench] matrix on device in {time.time() - t0:.1f}s: slots {info_m['slots']} "
        f"({'one triangle, ' if sym else ''}padding {info_m['slots'] / nval - 1:.4f}), "
        f"{info_m['shared_slices']} of "
        f"{info_m['slices']} slices with shared offsets, {info_m['device_bytes'] / 1e9:.2f} GB")
    t_create = time.time() - t0
    b = torch.from_numpy(b_np).to(dev)
    # setup, outside the timed region: the basis interval estimated on the
    # device from the same start vector as the host estimate the solves use
    v0 = torch.from_numpy(si_start_vector(A.n)).to(dev)
    P.interval(M, v0, method="lanczos", steps=20)
    torch.cuda.synchronize()
    t0 = time.time()
    est = P.interval(M, v0, method="lanczos", steps=20)
    setup = {"matrix_create_s": t_create, "interval_device_ms": 1e3 * (time.time() - t0),
             "interval_device": list(est["interval"]),
             "interval_device_vs_host": max(abs(est["interval"][i] - interval[i]) / interval[i]
                                            for i in (0, 1))}
    log(f"[bench] device Lanczos interval {est['interval']} in "
        f"{setup['interval_device_ms']:.1f} ms (relative difference from the host estimate "
        f"{setup['interval_device_vs_host']:.1e})")
    if args.mode == "kernels":
        print(json.dumps(kernel_pass(P, torch, M, A, b, interval, args, col_frac, nval)),
              flush=True)
        return 0
    opts = dict(s=args.s, sweeps=args.sweeps, interval=interval, tol=args.tol,
                profile=not args.no_profile)

    def step():
        x64, i64 = P.solve(M, b, **opts)
        imx = None
        if not args.no_mixed:
            _, imx = P.solve(M, b, precision="mixed", **opts)
        return x64, i64, imx

    for w in range(args.warmup):
        _, i64, imx = step()
        log(f"[bench] warmup {w}: fp64 {i64['device_ms']:.1f} ms {i64['outer_iters']} outer "
            f"{i64['status_name']}" + ("" if imx is None else
                                       f"; mixed {imx['device_ms']:.1f} ms "
                                       f"{imx['refinements']} refinements"))
    torch.cuda.synchronize()
    recs = []
    t_start = time.time()
    for k in range(args.steps):
        torch.cuda.synchronize()
        ts = time.time()
        x64, i64, imx = step()
        torch.cuda.synchronize()
        recs.append((time.time() - ts, i64, imx))
        log(f"[bench] step {k}: wall {recs[-1][0]:.3f}s fp64 {i64['device_ms']:.1f} ms "
            f"({i64['outer_iters']} outer, relres {i64['relres']:.2e})"
            + ("" if imx is None else f", mixed {imx['device_ms']:.1f} ms "
               f"({imx['refinements']} refinements, {imx['outer_iters']} inner)"))
    torch.cuda.synchronize()
    total = time.time() - t_start

    fp64_s = float(np.median([r[1]["device_ms"] for r in recs])) / 1e3
    last = recs[-1][1]
    n, nnz, s = A.n, A.nnz, args.s
    out = {
        "metric": METRIC, "value": fp64_s, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": False, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"27-point variable-coefficient diffusion {args.N}^3, "
                               "log-uniform k in [1e-2,1e2] on 8^3 blocks, b~N(0,1), Jacobi",
                   "n": n, "nnz": nnz, "s": s, "sweeps": args.sweeps, "tol": args.tol,
                   "interval": list(interval), "layout_slots": info_m["slots"],
                   "symmetric_storage": sym},
        "fp64": {"time_s": fp64_s, "outer_iters": last["outer_iters"], "relres": last["relres"],
                 "status": last["status_name"],
                 "ms_per_outer_iter": 1e3 * fp64_s / max(last["outer_iters"], 1)},
    }
    if not args.no_mixed:
        mx_s = float(np.median([r[2]["device_ms"] for r in recs])) / 1e3
        lm = recs[-1][2]
        # the iteration counts with two FGS sweeps move with rounding (see
        # --mode seeds); the time per iteration does not
        per_inner = 1e3 * mx_s / max(lm["outer_iters"], 1)
        out["mixed"] = {"time_s": mx_s, "refinements": lm["refinements"],
                        "inner_iters": lm["outer_iters"], "relres_true": lm["relres"],
                        "speedup_vs_fp64": fp64_s / mx_s, "status": lm["status_name"],
                        "ms_per_inner_iter": per_inner,
                        "speedup_per_iteration": out["fp64"]["ms_per_outer_iter"] / per_inner}
    if not args.no_profile:
        pr = last["profile"]
        sp = pr["spmv"]
        # algorithmic bytes of one SpMV launch of the matrix powers kernel:
        # what the stored format has to move (8 B per stored value -- no
        # column indices, one triangle plus the diagonal with the symmetric
        # half storage -- x read, y written, the epilogue's vectors), averaged
        # over the s launches.  The same work on a CSR stream (12 B per
        # nonzero, 4 B per row pointer) is reported beside it as a
        # CSR-equivalent rate, never as the roofline figure.
        b_fmt = spmv_family_bytes(n, nval, s, 8, col_frac, dinv_read=not sym) / s
        b_csr = csr_family_bytes(n, nnz, s, 8) / s
        t_launch = sp["ms"] / 1e3 / sp["launches"]
        achieved = b_fmt / t_launch / 1e9
        traffic = counter_traffic() if (args.N == 192 and s == 6) else None
        triad = triad_peak(P, torch, dev)
        out["roofline"] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                           "kernel": "k_spmv (matrix powers kernel, FP64)",
                           "avg_launch_us": 1e6 * t_launch, "bytes_per_launch": b_fmt,
                           "bytes_model": "stored format: 8 B per stored value (diagonal and "
                                          "upper triangle), 8 B per vector element read or "
                                          "written (x, y, epilogue z vectors)",
                           "achievable_peak": {"triad_gbs": triad["gbs"],
                                               "frac_of_triad": achieved / triad["gbs"],
                                               "triad_bytes": triad["bytes"],
                                               "kernel": "sspcg_stream_triad"},
                           "csr_equivalent": {"bytes_per_launch": b_csr,
                                              "gbs": b_csr / t_launch / 1e9},
                           "traffic_gbs": None if traffic is None else traffic / t_launch / 1e9}
        pb = phase_bytes(n, s, 8)
        phases = {}
        tot_f, tot_ms = 0.0, 0.0
        for ph in ("spmv", "gram_update", "gram_rect", "xr"):
            e = pr[ph]
            if e["launches"] == 0:
                continue
            nf = (b_fmt if ph == "spmv" else pb[ph]) * e["launches"]
            phases[ph] = {"launches": e["launches"], "ms": e["ms"],
                          "gbs": nf / (e["ms"] / 1e3) / 1e9}
            if ph == "spmv":
                phases[ph]["csr_equivalent_gbs"] = b_csr * e["launches"] / (e["ms"] / 1e3) / 1e9
            tot_f += nf
            tot_ms += e["ms"]
        for ph in ("fgs", "norm"):
            phases[ph] = {"launches": pr[ph]["launches"], "ms": pr[ph]["ms"]}
        out["phases"] = phases
        sg = [p for p in ("spmv", "gram_update", "gram_rect") if p in phases]
        ms_sg = sum(phases[p]["ms"] for p in sg)
        gbs_sg = sum(phases[p]["gbs"] * phases[p]["ms"] for p in sg) / ms_sg
        out["hbm_gbs_spmv_gram"] = gbs_sg
        out["spmv_gram_frac_of_peak"] = gbs_sg / HBM_PEAK_GBS
        out["spmv_gram_frac_of_triad"] = gbs_sg / triad["gbs"]
        out["hbm_gbs_all_streaming"] = tot_f / (tot_ms / 1e3) / 1e9
        out["profiled_ms_total"] = sum(pr[p]["ms"] for p in L_PHASES)
    if not args.no_profile:
        # the same FP64 solve without the per-phase events (their cost)
        _, iu = P.solve(M, b, s=args.s, sweeps=args.sweeps, interval=interval, tol=args.tol)
        out["fp64"]["time_s_without_phase_events"] = iu["device_ms"] / 1e3
    # and replayed from HIP graphs of check_every outer iterations (fewer launches)
    with torch.cuda.stream(torch.cuda.Stream(device=dev)):
        P.solve(M, b, s=args.s, sweeps=args.sweeps, interval=interval, tol=args.tol, graph=True)
        _, ig = P.solve(M, b, s=args.s, sweeps=args.sweeps, interval=interval, tol=args.tol,
                        graph=True)
    torch.cuda.synchronize()
    out["fp64"]["time_s_graph_replay"] = ig["device_ms"] / 1e3
    out["fp64"]["outer_iters_graph_replay"] = ig["outer_iters"]
    # the same solve with b uploaded from pinned host memory and x returned
    # there inside the timed region: the PCIe-inclusive time (the boundary
    # takes device buffers, so this is never `value`)
    bh = torch.from_numpy(b_np).pin_memory()
    xh = torch.empty_like(bh).pin_memory()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    bd = bh.to(dev, non_blocking=True)
    xd, ih = P.solve(M, bd, s=args.s, sweeps=args.sweeps, interval=interval, tol=args.tol)
    xh.copy_(xd, non_blocking=True)
    e1.record()
    torch.cuda.synchronize()
    out["fp64"]["time_s_pcie_inclusive"] = e0.elapsed_time(e1) / 1e3
    out["fp64"]["pcie_ms"] = e0.elapsed_time(e1) - ih["device_ms"]
    del bh, xh, bd, xd
    # the precision form's own target (outside the timed steps): mixed
    # refinement and FP64 to a relative residual of 1e-10, each with its
    # error against the oracle's reference solution of this system
    if args.N == 192 and s == 6 and args.sweeps == 2:
        out["to_1e-10_vs_oracle"] = accuracy_vs_oracle(P, M, b, A, b_np, interval, args,
                                                       with_mixed=not args.no_mixed)
    # the same system with other Gram solves (outside the timed steps): the
    # exact Cholesky solve and adaptive FGS sweeps (stop once
    # ||m - W a|| <= 1e-3 ||m||, at most 30), FP64 and mixed
    variants = {}
    for name, kw in (("cholesky", dict(sweeps=1, gram="cholesky")),
                     ("fgs_adaptive_1e-3", dict(sweeps=30, sweep_tol=1e-3))):
        variants[name] = {}
        for prec in ("fp64",) + (() if args.no_mixed else ("mixed",)):
            _, iv = P.solve(M, b, s=args.s, interval=interval, tol=args.tol, precision=prec, **kw)
            variants[name][prec] = {"time_s": iv["device_ms"] / 1e3, "status": iv["status_name"],
                                    "outer_iters" if prec == "fp64" else "inner_iters":
                                        iv["outer_iters"]}
    out["gram_solve_variants"] = variants
    # classical PCG comparator on the same system (outside the timed steps)
    _, ip = P.pcg(M, b, tol=args.tol)
    out["pcg"] = {"time_s": ip["device_ms"] / 1e3, "iters": ip["outer_iters"],
                  "relres": ip["relres"]}
    out["setup"] = setup
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle) ...")
        per_outer = (csr_family_bytes(n, nnz, s, 8)
                     + sum(v for k, v in phase_bytes(n, s, 8).items()))
        out["cpu_baseline"] = cpu_baseline(A, b_np, interval, s, args.sweeps,
                                           last["outer_iters"], args.cpu_sample_outer, per_outer)
    print(json.dumps(out), flush=True)
    return 0


L_PHASES = ["spmv", "gram_update", "gram_rect", "fgs", "norm", "xr"]

COPY_BYTES = 1 << 30   # calibration copy: 1 GiB read + 1 GiB written
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_k_spmv_27pt_192.json")


def code_digest(files) -> str:
    """SHA-256 of the code of the given C/HIP sources: comments removed and
    whitespace collapsed, so that only a change of the code itself marks a
    counter record as stale."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in files:
        s = open(os.path.join(ROOT, f), encoding="utf-8").read()
        s = re.sub(r"/\*.*?\*/", " ", s, flags=re.S)
        s = re.sub(r"//[^\n]*", " ", s)
        h.update(" ".join(s.split()).encode())
        h.update(b"\0")
    return h.hexdigest()


def counter_traffic():
    """HBM bytes per SpMV launch measured by rocprofv3 counters (FETCH_SIZE,
    WRITE_SIZE, scaled by a copy of known size), from the committed record --
    or None when the code of the SpMV sources changed since the counters were
    taken."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
        if code_digest(rec["sources"]) != rec["source_code_sha256"]:
            return None
        return rec["traffic_bytes_per_launch"]
    except (OSError, KeyError, ValueError):
        return None


RECORDS = os.path.join(ROOT, "tests", "golden", "solutions")


def oracle_record(case: str, A, b):
    """The oracle's committed solution record of this system (written by
    tests/golden/make_solution_records.py from the CPU oracle alone), or None
    when it is missing or was made for other inputs."""
    import sspcg_inputs as si
    try:
        rec = json.load(open(os.path.join(RECORDS, case + ".json")))
    except (OSError, ValueError):
        return None
    if rec["n"] != A.n or rec["digest_val"] != si.digest(A.val) or rec["digest_b"] != si.digest(b):
        return None
    return rec


def error_vs_record(x, rec) -> dict:
    """Relative error of the device solution x against an oracle record: the
    2-norm error estimated from the record's uniformly sampled entries
    (sqrt(n/k * sum of squared sampled differences) / ||x_oracle||), the
    largest sampled difference over the largest sampled |x_oracle|, and the
    difference of the norms."""
    import torch
    import sspcg_inputs as si
    idx = si.sample_indices(rec["n"], rec["n_samples"])
    xs = x[torch.from_numpy(idx).to(x.device)].cpu().numpy()
    xo = np.asarray(rec["x_samples"])
    d = xs - xo
    nx = torch.linalg.vector_norm(x).item()
    return {"rel_error_sampled": float(np.sqrt(rec["n"] / idx.size * np.sum(d * d))
                                       / rec["norm_x"]),
            "max_sampled_diff_rel": float(np.abs(d).max() / np.abs(xo).max()),
            "norm_rel_diff": abs(nx - rec["norm_x"]) / rec["norm_x"],
            "samples": int(idx.size), "oracle": rec["what"], "oracle_tol": rec["tol"],
            "oracle_iters": rec["iters"], "record": rec["case"]}


def accuracy_vs_oracle(P, M, b, A, b_np, interval, args, with_mixed=True) -> dict:
    """The precision form's target on the benchmark system: mixed refinement
    and FP64 s-step PCG, each to a relative residual of 1e-10, with their
    errors against x_ref, the oracle's classical PCG solution to 1e-13 (a
    committed record)."""
    ref = oracle_record("diffusion27_192_pcg", A, b_np)
    out = {"x_ref": None if ref is None else {"record": ref["case"], "what": ref["what"],
                                               "tol": ref["tol"], "iters": ref["iters"]}}
    opts = dict(s=args.s, sweeps=args.sweeps, interval=interval, tol=1e-10)
    x8, i8 = P.solve(M, b, **opts)
    out["fp64"] = {"time_s": i8["device_ms"] / 1e3, "outer_iters": i8["outer_iters"],
                   "relres": i8["relres"], "relres_true": i8["relres_true"],
                   "status": i8["status_name"],
                   "error_vs_x_ref": None if ref is None else error_vs_record(x8, ref)}
    del x8
    if with_mixed:
        xm, im = P.solve(M, b, precision="mixed", **opts)
        out["mixed"] = {"time_s": im["device_ms"] / 1e3, "refinements": im["refinements"],
                        "inner_iters": im["outer_iters"], "relres_true": im["relres_true"],
                        "status": im["status_name"],
                        "error_vs_x_ref": None if ref is None else error_vs_record(xm, ref)}
        out["mixed_speedup_vs_fp64"] = i8["device_ms"] / im["device_ms"]
    log(f"[bench] to 1e-10: {out}")
    return out


TRAFFIC_SOURCES = ["paper_2603_09790_amd/csrc/sell.hip", "paper_2603_09790_amd/csrc/common.h"]


def counter_dispatches(outdir: str, counter: str) -> list:
    """(kernel short name, value) of `counter` for every dispatch in the
    rocprofv3 database(s) (*_results.db, SQLite) under outdir."""
    import glob
    import sqlite3
    files = glob.glob(os.path.join(outdir, "**", "*_results.db"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no rocprofv3 *_results.db under {outdir}")
    out = []
    for f in files:
        con = sqlite3.connect(f)
        q = ("select dispatch_id, kernel_name, sum(value) from counters_collection "
             "where counter_name = ? group by dispatch_id, kernel_name")
        out += [(short_kernel_name(name), float(v)) for _, name, v in con.execute(q, (counter,))]
        con.close()
    return out


def trace_summary(outdir: str, min_pct: float = 0.01) -> str:
    """Markdown table of a rocprofv3 kernel trace (*_results.db under
    outdir): calls, total, average, min and max duration per kernel."""
    import glob
    import sqlite3
    files = glob.glob(os.path.join(outdir, "**", "*_results.db"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no rocprofv3 *_results.db under {outdir}")
    per = {}
    for f in files:
        con = sqlite3.connect(f)
        for name, dur in con.execute("select name, duration from kernels"):
            per.setdefault(short_kernel_name(name), []).append(float(dur))
        con.close()
    total = sum(sum(v) for v in per.values())
    lines = ["| kernel | calls | total ms | avg us | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|"]
    for k, v in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        pct = 100.0 * sum(v) / total
        if pct < min_pct:
            continue
        lines.append(f"| `{k}` | {len(v)} | {sum(v) / 1e6:.2f} | {np.mean(v) / 1e3:.1f} | "
                     f"{min(v) / 1e3:.1f} | {max(v) / 1e3:.1f} | {pct:.2f} |")
    return "\n".join(lines)


UNIT_KERNELS = ["k_spmv<double, 0>", "k_spmv<double, 1>", "k_spmv<double, 2>",
                "k_spmv<float, 0>", "k_update_gram<6, double, 1, 1>", "k_gram_rect<6, double, 2>",
                "k_xr<6, double, 2>"]


def units_summary(k1_dir: str, k2_dir: str) -> str:
    """Markdown table of the unit counters of the hot kernels (two passes over
    --mode kernels).  Fractions are unit-busy cycles over the kernel's cycles
    (SQ_CYCLES per shader engine, 32 engines) and the 256 CUs' units; counts
    are per wavefront."""
    c = {}
    for d, names in ((k1_dir, ["TA_TA_BUSY_sum", "TA_ADDR_STALLED_BY_TC_CYCLES_sum",
                               "TCP_PENDING_STALL_CYCLES_sum", "TCP_TCC_READ_REQ_sum"]),
                     (k2_dir, ["TCC_HIT_sum", "TCC_MISS_sum", "SQ_CYCLES", "SQ_WAVES",
                               "SQ_INSTS_VMEM_RD", "SQ_INSTS_LDS", "SQ_INSTS_VALU"])):
        for nm in names:
            for k, v in counter_rows(d, nm).items():
                c.setdefault(k, {})[nm] = v
    cus, ses = 256, 32
    lines = ["| kernel | TA busy | TA stalled by L1 | L1 pending-miss stall | vector-memory loads / wave "
             "| LDS instr / wave | VALU / wave | L2 hit rate |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for k in UNIT_KERNELS:
        v = c.get(k)
        if not v or "SQ_CYCLES" not in v or "TA_TA_BUSY_sum" not in v:
            continue
        cyc = v["SQ_CYCLES"] / ses
        waves = max(v["SQ_WAVES"], 1.0)
        hit = v["TCC_HIT_sum"] / max(v["TCC_HIT_sum"] + v["TCC_MISS_sum"], 1.0)
        lines.append(f"| `{k}` | {v['TA_TA_BUSY_sum'] / cus / cyc:.2f} | "
                     f"{v['TA_ADDR_STALLED_BY_TC_CYCLES_sum'] / max(v['TA_TA_BUSY_sum'], 1):.2f} | "
                     f"{v['TCP_PENDING_STALL_CYCLES_sum'] / cus / cyc:.2f} | "
                     f"{v['SQ_INSTS_VMEM_RD'] / waves:.1f} | {v['SQ_INSTS_LDS'] / waves:.1f} | "
                     f"{v['SQ_INSTS_VALU'] / waves:.0f} | {hit:.2f} |")
    return "\n".join(lines)


def counter_rows(outdir: str, counter: str) -> dict:
    """Per kernel, the mean value of `counter` per dispatch; for the device
    copy (several sizes in one run) the largest dispatch, the 1 GiB copy."""
    vals = {}
    for name, v in counter_dispatches(outdir, counter):
        vals.setdefault(name, []).append(v)
    return {k: float(max(v) if "copyBuffer" in k else np.mean(v)) for k, v in vals.items()}


def short_kernel_name(full: str) -> str:
    """'void sspcg::(anonymous namespace)::k_spmv<double, 0>(...)' -> 'k_spmv<double, 0>'."""
    import re
    m = re.search(r"\b(k_\w+(?:<[^()]*?>)?)\s*\(", full) or re.search(r"\b(k_\w+(?:<[^()]*?>)?)", full)
    if m:
        return m.group(1)
    return "__amd_rocclr_copyBuffer" if "copyBuffer" in full else full


def traffic_record(fetch_dir: str, write_dir: str, s: int) -> dict:
    """HBM-side bytes per SpMV launch of the matrix powers kernel from the
    FETCH_SIZE and WRITE_SIZE passes (KiB per dispatch) over --mode kernels,
    each scaled by what the same counter reads for the 1 GiB device copy of
    that run; written to profiles/ with a digest of the SpMV sources' code."""
    fetch = counter_rows(fetch_dir, "FETCH_SIZE")
    write = counter_rows(write_dir, "WRITE_SIZE")
    ck = "__amd_rocclr_copyBuffer"     # largest dispatch: the 1 GiB calibration copy
    if ck not in fetch or ck not in write:
        raise RuntimeError("the counter passes hold no device copy to calibrate with")
    fscale = COPY_BYTES / (fetch[ck] * 1024.0)
    wscale = COPY_BYTES / (write[ck] * 1024.0)
    modes = {}
    for k in fetch:
        if k.startswith("k_spmv<double"):
            mode = k.split(",")[1].strip().rstrip(">").strip()
            name = f"k_spmv<double, {mode}>"
            modes[name] = {"fetch_kib": fetch[k], "write_kib": write.get(k, 0.0),
                           "traffic_bytes": fetch[k] * 1024.0 * fscale
                           + write.get(k, 0.0) * 1024.0 * wscale}
    need = ["k_spmv<double, 0>", "k_spmv<double, 1>", "k_spmv<double, 2>"]
    if any(m not in modes for m in need):
        raise RuntimeError(f"counter passes lack SpMV modes: found {sorted(modes)}")
    per_launch = (modes[need[1]]["traffic_bytes"] + (s - 2) * modes[need[2]]["traffic_bytes"]
                  + modes[need[0]]["traffic_bytes"]) / s
    rec = {"kernel": "k_spmv (matrix powers kernel, FP64)",
           "workload": f"27-point diffusion 192^3, s = {s}",
           "source_code_sha256": code_digest(TRAFFIC_SOURCES), "sources": TRAFFIC_SOURCES,
           "calibration": {"kernel": ck + " (1 GiB device copy)", "bytes_each_way": COPY_BYTES,
                           "fetch_kib": fetch[ck], "write_kib": write[ck],
                           "fetch_scale": fscale, "write_scale": wscale},
           "modes": modes, "traffic_bytes_per_launch": per_launch,
           "note": "average over the s launches of one matrix powers kernel: modes 1, "
                   "(s-2) x 2 and 0",
           "commands": [
               "export TMPDIR=/tmp; timeout -s KILL 180 rocprofv3 --pmc FETCH_SIZE -d "
               "gpurun_out/pmc_FETCH_SIZE -o kern -- python3 bench.py --mode kernels --reps 2",
               "export TMPDIR=/tmp; timeout -s KILL 180 rocprofv3 --pmc WRITE_SIZE -d "
               "gpurun_out/pmc_WRITE_SIZE -o kern -- python3 bench.py --mode kernels --reps 2",
               "python3 bench.py --mode traffic-record"]}
    with open(TRAFFIC_RECORD, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def seed_spread(P, torch, dev, args, nseeds=5):
    """FP64 and mixed solves of the 192^3 system for nseeds right-hand sides
    b ~ N(0,1) (the benchmark's seed and the next ones): iteration counts and
    times to tolerance, whose spread shows how much of a single run's count
    is rounding-driven."""
    import sspcg_inputs as si
    A, _, interval = build_workload(args.N)
    M = P.Matrix.from_csr(A, fp32=True, device=dev)
    opts = dict(s=args.s, sweeps=args.sweeps, interval=interval, tol=args.tol)
    runs = []
    for k in range(nseeds):
        b = torch.from_numpy(si.rhs_normal(A.n, si.SEED_RHS + k)).to(dev)
        if k == 0:
            P.solve(M, b, **opts)   # warm-up
        _, i64 = P.solve(M, b, **opts)
        _, imx = P.solve(M, b, precision="mixed", **opts)
        r = {"seed": si.SEED_RHS + k, "fp64_s": i64["device_ms"] / 1e3,
             "fp64_outer": i64["outer_iters"], "fp64_status": i64["status_name"],
             "mixed_s": imx["device_ms"] / 1e3, "mixed_inner": imx["outer_iters"],
             "mixed_refinements": imx["refinements"], "mixed_status": imx["status_name"],
             "speedup": i64["device_ms"] / imx["device_ms"]}
        runs.append(r)
        log(f"[seeds] {r}")

    def stats(key):
        v = np.array([r[key] for r in runs], dtype=float)
        return {"mean": float(v.mean()), "min": float(v.min()), "max": float(v.max())}

    return {"mode": "seeds", "workload": f"27-point variable-coefficient diffusion {args.N}^3",
            "s": args.s, "sweeps": args.sweeps, "tol": args.tol, "runs": runs,
            **{k: stats(k) for k in ("fp64_s", "fp64_outer", "mixed_s", "mixed_inner", "speedup")}}


def oracle_times_small(w, gpu_outer, reps=3):
    """The oracle's 2D Poisson 64^2 solve (s = 4, nu = 2, 1e-8) on one host
    thread and on all of them: median wall time of `reps` solves each."""
    import oracle
    oracle.build()
    full = os.cpu_count() or 1
    out = {"host": host_description(), "gpu_outer_iters": gpu_outer}
    for k in (1, full):
        oracle.set_threads(k)
        ts = []
        for _ in range(reps):
            t0 = time.time()
            _, r = oracle.sspcg(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-8)
            ts.append(time.time() - t0)
        out[f"threads_{k}"] = {"seconds": float(np.median(ts)), "outer_iters": r["iters"]}
    oracle.set_threads(full)
    return out


def oracle_per_outer(w, gpu_outer, sample=10):
    """The oracle's 7-point 128^3 s = 4, nu = 2 iteration on one host thread
    and on all of them: seconds per outer iteration from the difference of a
    (2 + sample)- and a 2-iteration run (setup excluded), and that times the
    GPU's outer-iteration count."""
    import oracle
    oracle.build()
    full = os.cpu_count() or 1
    out = {"host": host_description(), "gpu_outer_iters": gpu_outer, "sample_outer": sample}
    for k in (1, full):
        oracle.set_threads(k)
        ts = []
        for m in (2, 2 + sample):
            t0 = time.time()
            oracle.sspcg(w["A"], w["b"], s=4, sweeps=2, interval=w["interval"], tol=1e-30,
                         max_outer=m)
            ts.append(time.time() - t0)
        per = (ts[1] - ts[0]) / sample
        out[f"threads_{k}"] = {"seconds_per_outer": per, "scaled_to_gpu_count": per * gpu_outer}
    oracle.set_threads(full)
    return out


def other_configs(P, torch, dev, args):
    """Times the other standard workloads (their parity is in the tests):
    2D Poisson 64^2 (launch-latency bound), 7-point Poisson 128^3 over s and
    sweeps, the mixed form to 1e-10 on the 192^3 benchmark system, and the
    differentiable solve (forward + backward) on 7-point diffusion 96^3."""
    import sspcg_inputs as si
    out = {}
    # 2D Poisson 64^2, s = 4, two sweeps, closed-form interval
    w = si.workload("poisson5")
    M = P.Matrix.from_csr(w["A"], device=dev)
    b = torch.from_numpy(w["b"]).to(dev)
    res = {}
    stream = torch.cuda.Stream()
    for name, fn in (("sspcg", lambda: P.solve(M, b, s=4, sweeps=2, interval=w["interval"], tol=1e-8)),
                     ("sspcg_graph", lambda: P.solve(M, b, s=4, sweeps=2, interval=w["interval"],
                                                     tol=1e-8, graph=True, check_every=16)),
                     ("pcg", lambda: P.pcg(M, b, tol=1e-8))):
        with torch.cuda.stream(stream):
            fn()
            ts = [fn()[1] for _ in range(3)]
        res[name] = {"time_ms": float(np.median([t["device_ms"] for t in ts])),
                     "iters": ts[-1]["outer_iters"]}
        res[name]["us_per_iter"] = 1e3 * res[name]["time_ms"] / max(res[name]["iters"], 1)
    out["poisson5_64"] = res
    log(f"[configs] poisson5 64^2: {res}")
    out["poisson5_64"]["oracle"] = oracle_times_small(w, res["sspcg"]["iters"])
    log(f"[configs] poisson5 64^2 oracle: {out['poisson5_64']['oracle']}")
    # 7-point Poisson 128^3 grid of s and sweeps
    w = si.workload("poisson7")
    M = P.Matrix.from_csr(w["A"], device=dev)
    b = torch.from_numpy(w["b"]).to(dev)
    grid = {}
    _, ip = P.pcg(M, b, tol=1e-8)
    grid["pcg"] = {"time_ms": ip["device_ms"], "iters": ip["outer_iters"]}
    for s_ in (2, 4, 6, 8):
        for nu in (1, 2, 3):
            _, i = P.solve(M, b, s=s_, sweeps=nu, interval=w["interval"], tol=1e-8)
            grid[f"s{s_}_nu{nu}"] = {"time_ms": i["device_ms"], "outer_iters": i["outer_iters"],
                                     "status": i["status_name"]}
    out["poisson7_128"] = {"interval": list(w["interval"]), "runs": grid}
    log(f"[configs] poisson7 128^3: {grid}")
    out["poisson7_128"]["oracle_s4_nu2"] = oracle_per_outer(w, grid["s4_nu2"]["outer_iters"])
    log(f"[configs] poisson7 128^3 oracle: {out['poisson7_128']['oracle_s4_nu2']}")
    # mixed and FP64 to 1e-10 on the benchmark system, errors against the
    # oracle's reference solution (classical PCG to 1e-13, a committed record)
    A, b_np, interval = build_workload(192)
    M = P.Matrix.from_csr(A, fp32=True, device=dev)
    b = torch.from_numpy(b_np).to(dev)
    cargs = argparse.Namespace(s=6, sweeps=2)
    out["diffusion27_192_to_1e-10"] = accuracy_vs_oracle(P, M, b, A, b_np, interval, cargs)
    log(f"[configs] diffusion27 192^3 to 1e-10: {out['diffusion27_192_to_1e-10']}")
    del M
    # differentiable solve, 7-point diffusion 96^3
    w = si.workload("diffusion7")
    A = w["A"]
    M = P.Matrix.from_csr(A, device=dev)
    theta = torch.from_numpy(w["theta"]).to(dev).requires_grad_(True)
    b = torch.from_numpy(w["b"]).to(dev)
    xt = torch.from_numpy(w["x_target"]).to(dev)
    opts = dict(s=4, sweeps=2, interval=w["interval"], tol=1e-8)
    for rep in range(2):
        theta.grad = None
        torch.cuda.synchronize()
        t0 = time.time()
        x = P.DiffusionSolve.apply(theta, b, M, opts)
        loss = 0.5 * torch.sum((x - xt) ** 2)
        torch.cuda.synchronize()
        t1 = time.time()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.time()
    # the two solves inside: forward A x = b, adjoint A lambda = x - x_target
    # (the matrix holds A(theta) from the step above)
    _, i_f = P.solve(M, b, **opts)
    _, i_b = P.solve(M, (x.detach() - xt).contiguous(), **opts)
    out["diffusion7_96_grad"] = {"forward_s": t1 - t0, "backward_s": t2 - t1,
                                 "forward_solve": {"outer_iters": i_f["outer_iters"],
                                                   "device_ms": i_f["device_ms"]},
                                 "adjoint_solve": {"outer_iters": i_b["outer_iters"],
                                                   "device_ms": i_b["device_ms"]},
                                 "loss": loss.item(),
                                 "grad_norm": torch.linalg.vector_norm(theta.grad).item()}
    log(f"[configs] diffusion7 96^3 gradient: {out['diffusion7_96_grad']}")
    return out


def paper_experiments(P, torch, dev, args):
    """The paper's Gram-solve experiments (Sec. 3.4 and its residual-history
    comparison) on one GPU's share of its weak-scaling workload: the
    constant-coefficient 27-point matrix as in HPCG on N^3 (N = 200 per GPU
    in the paper), unit right-hand side, lambda_min = 0 and a power-method
    lambda_max (Sec. 2), tolerance 1e-8.

    For s in {4, 6}: FGS with 30 and 60 sweeps and the Cholesky Gram solve,
    recording per outer iteration the relative residual and the reduced-system
    residuals eta_alpha, eta_beta; classical PCG with its residual sampled
    every s steps for the aligned comparison.
    """
    import sspcg_inputs as si
    N = args.paper_N
    t0 = time.time()
    A = si.hpcg27(N)
    b_np = np.ones(A.n)
    interval = si.power_bounds(A)
    log(f"[paper] 27pt HPCG {N}^3: n={A.n} nnz={A.nnz}, power-method interval {interval} "
        f"({time.time() - t0:.1f}s)")
    M = P.Matrix.from_csr(A, device=dev)
    b = torch.from_numpy(b_np).to(dev)
    v0 = torch.from_numpy(si.start_vector(A.n)).to(dev)
    torch.cuda.synchronize()
    t0 = time.time()
    pw = P.interval(M, v0, method="power", steps=50, rtol=1e-3)
    pw_ms = 1e3 * (time.time() - t0)
    log(f"[paper] device power method: {pw['interval']} after {pw['steps']} steps, "
        f"{pw_ms:.1f} ms")
    tol = 1e-8
    _, ip = P.pcg(M, b, tol=tol, history=True)
    hp = ip["history"]
    runs, summary = {}, {"workload": f"27-point Poisson (HPCG) {N}^3, b = 1, power-method interval",
                         "n": A.n, "nnz": A.nnz, "interval": list(interval), "tol": tol,
                         "pcg": {"iters": ip["outer_iters"], "time_s": ip["device_ms"] / 1e3},
                         "device_power_interval": {"interval": list(pw["interval"]),
                                                   "steps": pw["steps"], "ms": pw_ms}}
    for s in (4, 6):
        for gram, sweeps in (("fgs", 30), ("fgs", 60), ("cholesky", 1)):
            x, info = P.solve(M, b, s=s, sweeps=sweeps, gram=gram, interval=interval, tol=tol,
                              history=True)
            h = info["history"]
            k = np.arange(1, len(h) + 1)
            aligned = hp[np.minimum(k * s, len(hp)) - 1]
            name = f"s{s}_{gram}{sweeps if gram == 'fgs' else ''}"
            runs[name] = {"relres": h[:, 0].tolist(), "eta_alpha": h[:, 1].tolist(),
                          "eta_beta": h[:, 2].tolist(), "conjugacy_defect": h[:, 3].tolist(),
                          "pcg_every_s": aligned.tolist()}
            eb = h[:-1, 2] if len(h) > 1 else h[:, 2]
            summary[name] = {"outer_iters": info["outer_iters"], "krylov_steps": s * info["outer_iters"],
                             "time_s": info["device_ms"] / 1e3, "status": info["status_name"],
                             "eta_alpha_max": float(h[:, 1].max()), "eta_alpha_median": float(np.median(h[:, 1])),
                             "eta_beta_max": float(eb.max()), "eta_beta_median": float(np.median(eb)),
                             "conjugacy_defect_median": float(np.median(h[:-1, 3] if len(h) > 1 else h[:, 3])),
                             "max_log10_gap_to_pcg": float(np.max(np.abs(np.log10(h[:, 0]) - np.log10(aligned))))}
            log(f"[paper] {name}: {summary[name]}")
    return {"summary": summary, "runs": runs, "pcg_history": hp.tolist()}


def kernel_pass(P, torch, M, A, b, interval, args, col_frac, nval):
    """Launches each hot kernel `reps` times and a plain copy of known size.

    Times each kernel with events on the current stream (the one the library
    launches on).  Used under rocprofv3 --pmc to relate FETCH_SIZE and
    WRITE_SIZE to bytes: the copy moves exactly COPY_BYTES each way.
    """
    n, s, reps = A.n, args.s, args.reps
    ld = P.leading_dim(n)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device=M.device)
    dst = torch.empty_like(src)
    x = torch.randn(n, dtype=torch.float64, device=M.device)
    Zb = torch.randn((s, ld), dtype=torch.float64, device=M.device)
    Qb, AZb, AQb = torch.randn_like(Zb), torch.randn_like(Zb), torch.randn_like(Zb)
    beta = torch.randn((s, s), dtype=torch.float64, device=M.device) * 0.1
    alpha = torch.randn(s, dtype=torch.float64, device=M.device)
    r = torch.randn(n, dtype=torch.float64, device=M.device)
    xr_x = torch.zeros(n, dtype=torch.float64, device=M.device)
    z1 = torch.empty_like(xr_x)
    sym = bool(M.info()["symmetric"])
    ev = lambda: torch.cuda.Event(enable_timing=True)
    out = {}

    def timed(name, fn, nbytes):
        fn()
        torch.cuda.synchronize()
        a, z = ev(), ev()
        a.record()
        for _ in range(reps):
            fn()
        z.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(z) / reps
        out[name] = {"avg_ms": ms, "bytes": nbytes, "gbs": nbytes / (ms / 1e3) / 1e9}
        log(f"[kernels] {name}: {ms * 1e3:.1f} us, {out[name]['gbs']:.0f} GB/s")

    timed("copy_1GiB", lambda: dst.copy_(src), 2 * COPY_BYTES)
    timed("spmv_f64", lambda: P.spmv(M, x), spmv_bytes(n, nval, 8, col_frac))
    timed("mpk_f64_s%d" % s, lambda: P.mpk(M, r, s, interval, ld=ld),
          spmv_family_bytes(n, nval, s, 8, col_frac, dinv_read=not sym))
    timed("gram_update", lambda: P.block_update_gram(n, Zb, Qb, AZb, AQb, beta, r),
          (6 * s + 1) * 8 * n)
    timed("gram_rect", lambda: P.gram_rect(n, Qb, AZb), 2 * s * 8 * n)
    # as in the solve: z1 = M^{-1} r written as well
    timed("xr", lambda: P.xr_update(M, Qb, AQb, alpha, xr_x, r, z1), (2 * s + 6) * 8 * n)
    if M.fp32:
        x32 = x.float()
        timed("spmv_f32", lambda: P.spmv(M, x32), spmv_bytes(n, nval, 4, col_frac))
    return {"mode": "kernels", "n": n, "nnz": A.nnz, "s": s, "reps": reps, "kernels": out}

if __name__ == "__main__":
    sys.exit(main())
