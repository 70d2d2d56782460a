"""Planted mistakes in the oracle must fail its pins.

Each case copies the oracle's C source, plants one plausible mistake (a
dropped term, a wrong sign or index, a transposed operand, a wrong
coefficient), builds the copy with the oracle's own flags and runs the pin
tests against it in a child process (``SSPCG_ORACLE_LIB`` points the oracle
module at the copy).  The case passes when the pins fail.  Everything runs
on the CPU; the GPU library is not involved.
"""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "sspcg_oracle.c")
PINS64 = "tests/test_oracle_pins.py"
PINS32 = "tests/test_oracle_fp32_pins.py"

# (case, function whose body is changed, text in it, replacement, pin files)
MUTATIONS = [
    # Algorithm 2 (FP64)
    ("mpk: first step uses 2 alpha", "int basis, double* Z, double* P, int64_t ld)\n{",
     "ZP(2)[i] = al * PC(2)[i]", "ZP(2)[i] = 2.0 * al * PC(2)[i]", [PINS64]),
    ("mpk: gamma term dropped", "int basis, double* Z, double* P, int64_t ld)\n{",
     " - gm * ZP(q - 1)[i];", ";", [PINS64]),
    ("mpk: sigma sign", "int basis, double* Z, double* P, int64_t ld)\n{",
     "- 2.0 * sg * ZP(q)[i]", "+ 2.0 * sg * ZP(q)[i]", [PINS64]),
    # Gram blocks and updates of Algorithm 1 (FP64)
    ("gram: b1 from AQ", "void or_gram(", "b1[i] = or_dot(n, Q + (int64_t)i * ld, r);",
     "b1[i] = or_dot(n, AQ + (int64_t)i * ld, r);", [PINS64]),
    ("gram_rect: sign of B2", "void or_gram_rect(", "= -or_dot(", "= or_dot(", [PINS64]),
    ("block update: beta transposed", "void or_block_update(",
     "tq += q[l] * beta[l * s + j];", "tq += q[l] * beta[j * s + l];", [PINS64]),
    ("xr update: sign of the r update", "void or_xr_update(", "r[i] -= aqa;", "r[i] += aqa;",
     [PINS64]),
    # eq. fgs-iteration
    ("fgs: upper part dropped", "int or_fgs_tol(int s, int nrhs, const double* W, const double* B, int sweeps, double delta,\n               double* X)\n{",
     "for (int j = i + 1; j < s; ++j) t -=", "for (int j = s; j < s; ++j) t -=", [PINS64]),
    # FP32 storage pieces of the mixed form
    ("mpk_f32: gamma term dropped", "void or_mpk_f32(",
     "- gm * (double)ZP(q - 1)[i]);", ");", [PINS32]),
    ("mpk_f32: first step uses 2 alpha", "void or_mpk_f32(",
     "ZP(2)[i] = (float)(al * (double)PC(2)[i]", "ZP(2)[i] = (float)(2.0 * al * (double)PC(2)[i]",
     [PINS32]),
    ("mpk_f32: sigma sign at the first step", "void or_mpk_f32(",
     "- sg * (double)ZP(1)[i]", "+ sg * (double)ZP(1)[i]", [PINS32]),
    ("mpk_f32: Jacobi scaling dropped", "void or_mpk_f32(",
     "ZC(q + 1)[i] = (float)((double)dinv[i] * (double)ZP(q + 1)[i]);",
     "ZC(q + 1)[i] = ZP(q + 1)[i];", [PINS32]),
    ("spmv_f32: FP32 accumulation", "void or_spmv_f32(", "double acc = 0.0;",
     "float acc = 0.0f;", [PINS32]),
    ("gram_f32: b1 from AQ", "void or_gram_f32(", "b1[i] = dot_f32(n, Q + (int64_t)i * ld, r);",
     "b1[i] = dot_f32(n, AQ + (int64_t)i * ld, r);", [PINS32]),
    ("gram_rect_f32: sign of B2", "void or_gram_rect_f32(", "= -dot_f32(", "= dot_f32(", [PINS32]),
    ("block_update_f32: beta transposed", "void or_block_update_f32(",
     "tq += q[l] * beta[l * s + j];", "tq += q[l] * beta[j * s + l];", [PINS32]),
    ("block_update_f32: AQ updated from Q", "void or_block_update_f32(",
     "taq += aq[l] * beta[l * s + j];", "taq += q[l] * beta[l * s + j];", [PINS32]),
    ("block_update_f32: Z dropped", "void or_block_update_f32(",
     "(float)((double)Z[(int64_t)j * ld + i] + tq)", "(float)(tq)", [PINS32]),
    ("xr_update_f32: sign of the r update", "void or_xr_update_f32(",
     "r[i] = (float)((double)r[i] - aqa);", "r[i] = (float)((double)r[i] + aqa);", [PINS32]),
    ("xr_update_f32: x from AQ", "void or_xr_update_f32(",
     "qa += (double)Q[(int64_t)j * ld + i] * alpha[j];",
     "qa += (double)AQ[(int64_t)j * ld + i] * alpha[j];", [PINS32]),
    ("inner_f32: B2 from the wrong block", "int or_inner_sspcg_f32(",
     "or_gram_rect_f32(n, s, Q, P + ld, ld, B2);", "or_gram_rect_f32(n, s, Q, P, ld, B2);",
     [PINS32]),
    ("inner_f32: first AQ from P(:,1)", "int or_inner_sspcg_f32(",
     "memcpy(AQ, P + ld, sizeof(float) * n * s);", "memcpy(AQ, P, sizeof(float) * n * s);",
     [PINS32]),
    # differentiable form (chain rule through the assembly)
    ("theta grad: ghost term dropped", "void or_diffusion7_theta_grad(",
     "gtheta[i] += gd * (double)(6 - deg) * ki;", "(void)deg;", [PINS64]),
    ("theta grad: derivatives swapped", "void or_diffusion7_theta_grad(",
     "gtheta[i] -= gval[e] * dwi;", "gtheta[i] -= gval[e] * dwj;", [PINS64]),
]


def plant(src: str, anchor: str, old: str, new: str) -> str:
    """Replace the first `old` after `anchor` (which must occur once)."""
    assert src.count(anchor) == 1, anchor
    start = src.index(anchor)
    at = src.index(old, start)
    nxt = src.find("\n}\n", start)          # the mutation stays inside that function
    assert at < nxt, (anchor, old)
    return src[:at] + new + src[at + len(old):]


def run_case(tmp: str, k: int, case) -> tuple:
    name, anchor, old, new, pins = case
    with open(SRC) as f:
        src = plant(f.read(), anchor, old, new)
    cfile = os.path.join(tmp, f"m{k}.c")
    lib = os.path.join(tmp, f"m{k}.so")
    with open(cfile, "w") as f:
        f.write(src)
    subprocess.run(["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                    "-std=c99", "-w", "-o", lib, cfile, "-lm"], check=True)
    env = dict(os.environ, SSPCG_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *pins], cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=600)
    return name, r.returncode, r.stdout[-600:]


def test_planted_mistakes_fail_the_pins():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=4) as ex:
            results = list(ex.map(lambda kc: run_case(tmp, *kc), enumerate(MUTATIONS)))
    survived = [(name, rc, out) for name, rc, out in results if rc != 1]
    assert not survived, survived


def test_unmutated_copy_passes():
    """The harness itself: an unchanged copy, loaded the same way, passes."""
    with tempfile.TemporaryDirectory() as tmp:
        name, rc, out = run_case(tmp, 0, ("none", "void or_gram(", "b1[i]", "b1[i]",
                                          [PINS64, PINS32]))
    assert rc == 0, out
