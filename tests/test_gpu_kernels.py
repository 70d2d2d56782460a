"""Kernel-level parity of the HIP library against the CPU oracle.

Teacher forcing: the oracle's own states at outer iteration k (from
oracle_trace) are fed to each GPU kernel through the C ABI, and the GPU
output is compared with the oracle's next state.  Tolerances:
  * vectors of one kernel: |d| <= 1e-13 * max|ref| per column (FMA
    contraction and the MPK's M^{-1}-folded Chebyshev update differ from the
    oracle in rounding; measured <= 1.5e-14); one whole outer iteration:
    1e-12 (measured <= 2.7e-14);
  * Gram entries (W, b1, B2): |d_ij| <= 1e-12 * sum_r |Q_ri| |AQ_rj|, the
    forward-error scale of a dot product, since entries can cancel;
  * FP32 SpMV: bit-exact (same order, exact products, one rounding).
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_09790_amd as P
import sspcg_inputs as si
from oracle_trace import trace

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def gpu(a, dtype=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV, dtype=dtype)


def host(t):
    return t.detach().cpu().numpy()


def block(a, ld):
    """Oracle block (ncols, n) -> device tensor (ncols, ld), zero padded."""
    t = torch.zeros((a.shape[0], ld), dtype=torch.float64, device=DEV)
    t[:, :a.shape[1]] = gpu(a)
    return t


def col_close(got, ref, tol):
    got, ref = np.atleast_2d(got), np.atleast_2d(ref)
    for j in range(ref.shape[0]):
        scale = max(np.abs(ref[j]).max(), 1e-300)
        err = np.abs(got[j] - ref[j]).max()
        assert err <= tol * scale, f"column {j}: {err / scale:.3e} > {tol}"


def gram_close(got, ref, Q, AQ, tol=1e-12):
    scale = np.abs(Q) @ np.abs(AQ).T
    err = np.abs(got - ref)
    assert np.all(err <= tol * scale + 1e-300), f"max scaled err {np.max(err / scale):.3e}"


SYSTEMS = {
    # name: (kind, N, coefficients, storage) -- n values include ragged tails
    # (not multiples of 64); symmetric matrices are stored as one triangle
    # unless the storage is "full"
    "p5_64": ("5pt", 64, None, "auto"),
    "d7_13": ("7pt", 13, "theta", "auto"),
    "d27_17": ("27pt", 17, "blocks", "auto"),
    "p5_64_full": ("5pt", 64, None, "full"),      # uniform layout, both triangles
    "d7_13_full": ("7pt", 13, "theta", "full"),   # per-slice offset lists
    "d27_17_full": ("27pt", 17, "blocks", "full"),
}


def system(name):
    kind, N, coef, _ = SYSTEMS[name]
    n = N * N if kind == "5pt" else N**3
    kap = None
    if coef == "theta":
        kap = np.exp(si.theta_field(n))
    elif coef == "blocks":
        rng = np.random.default_rng(1)
        kap = 10.0 ** rng.uniform(-2, 2, n)
    A = si.stencil(kind, N, kap)
    b = si.rhs_normal(A.n)
    return A, b, si.lanczos_bounds(A)


@pytest.fixture(scope="module", params=list(SYSTEMS))
def sys_(request):
    A, b, interval = system(request.param)
    full = SYSTEMS[request.param][3] == "full"
    M = P.Matrix.from_csr(A, fp32=True, full_storage=full, device=DEV)
    assert M.info()["symmetric"] == (0 if full else 1)
    return A, b, interval, M


def test_spmv_fp64(sys_):
    A, _, _, M = sys_
    x = np.random.default_rng(5).normal(size=A.n)
    y = host(P.spmv(M, gpu(x)))
    ref = oracle.spmv(A, x)
    absA = A.__class__(A.n, A.row_ptr, A.col, np.abs(A.val), A.shape3)
    scale = oracle.spmv(absA, np.abs(x))
    assert np.all(np.abs(y - ref) <= 1e-14 * scale)


def test_spmv_fp32_bit_exact(sys_):
    A, _, _, M = sys_
    x32 = np.random.default_rng(6).normal(size=A.n).astype(np.float32)
    y = host(P.spmv(M, gpu(x32)))
    ref = oracle.spmv_f32(A, A.val.astype(np.float32), x32)
    assert np.array_equal(y, ref)


def test_spmv_unaligned_x_same_result(sys_):
    """x not 16-byte aligned: the LDS staging falls back to single-element
    loads (and the gathers are unaffected); the product is the same bits."""
    A, _, _, M = sys_
    x = np.random.default_rng(7).normal(size=A.n)
    buf = torch.zeros(A.n + 1, dtype=torch.float64, device=DEV)
    buf[1:] = gpu(x)
    xu = buf[1:]
    assert xu.data_ptr() % 16 == 8
    assert torch.equal(P.spmv(M, xu), P.spmv(M, gpu(x)))


def test_matrix_info_and_padding(sys_):
    A, _, _, M = sys_
    info = M.info()
    assert info["n"] == A.n and info["nnz"] == A.nnz
    if info["symmetric"]:
        # one triangle and the diagonal
        half = (A.nnz + A.n) // 2
        assert half <= info["slots"] <= 1.2 * half + 64 * 14
    else:
        assert A.nnz <= info["slots"] <= 1.2 * A.nnz + 64 * 27


@pytest.mark.parametrize("s", [1, 2, 4, 6, 8, 16])
def test_mpk(sys_, s):
    A, b, interval, M = sys_
    dinv = oracle.jacobi_inverse(A)
    r = np.random.default_rng(7).uniform(-1, 1, A.n)
    Zr, Pr = oracle.mpk(A, dinv, r, s, interval)
    ld = P.leading_dim(A.n)
    Z, Pm = P.mpk(M, gpu(r), s, interval, ld=ld)
    Z, Pm = host(Z)[:, :A.n], host(Pm)[:, :A.n]
    # T1: 1e-13 per column (measured <= 3.5e-15, also at s = 16)
    col_close(Z, Zr, 1e-13)
    col_close(Pm, Pr, 1e-13)
    assert np.array_equal(Pm[0], r)


def test_mpk_fp32(sys_):
    A, _, interval, M = sys_
    s = 4
    d = A.val.astype(np.float32)
    dinv32 = (1.0 / si.to_scipy(A).diagonal()).astype(np.float32)
    r32 = np.random.default_rng(8).uniform(-1, 1, A.n).astype(np.float32)
    Zr, Pr = oracle.mpk_f32(A, d, dinv32, r32, s, interval)
    Z, Pm = P.mpk(M, gpu(r32), s, interval)
    # FP32 storage: the GPU folds M^{-1} into the recurrence, the oracle keeps
    # zp; both round every stored vector to FP32
    col_close(host(Z), Zr.astype(np.float64), 2e-5)
    col_close(host(Pm), Pr.astype(np.float64), 2e-5)


@pytest.fixture(scope="module")
def traced():
    out = {}
    for name in SYSTEMS:
        A, b, interval = system(name)
        for s in (2, 6):
            _, _, states = trace(A, b, s=s, sweeps=2, interval=interval, tol=1e-14, max_outer=12)
            out[(name, s)] = (A, interval, states, P.Matrix.from_csr(A, device=DEV))
    return out


KEYS = [(n, s) for n in SYSTEMS for s in (2, 6)]


@pytest.mark.parametrize("key", KEYS)
def test_first_block_gram(traced, key):
    A, _, states, M = traced[key]
    st = states[0]
    ld = P.leading_dim(A.n)
    s = st["Z"].shape[0]
    Z, AZ = block(st["Z"], ld), block(st["P"][1:], ld)
    Q = torch.full_like(Z, float("nan"))
    AQ = torch.full_like(Z, float("nan"))
    r = gpu(st["P"][0])
    W, b1 = P.block_update_gram(A.n, Z, Q, AZ, AQ, None, r)
    assert torch.equal(Q[:, :A.n], Z[:, :A.n]) and torch.equal(AQ[:, :A.n], AZ[:, :A.n])
    gram_close(host(W), st["W"], st["Q"], st["AQ"])
    gram_close(host(b1)[:, None], st["b1"][:, None], st["Q"], st["r"][None, :])
    assert np.array_equal(host(W), host(W).T)


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("k", [0, 1, 5, 10])
def test_update_gram_and_rect(traced, key, k):
    A, _, states, M = traced[key]
    st, nx = states[k], states[k + 1]
    ld = P.leading_dim(A.n)
    Q, AQ = block(st["Q"], ld), block(st["AQ"], ld)
    Z, AZ = block(st["Znext"], ld), block(st["Pnext"][1:], ld)
    B2 = P.gram_rect(A.n, Q, AZ)
    gram_close(host(B2), st["B2"], st["Q"], st["Pnext"][1:])
    W, b1 = P.block_update_gram(A.n, Z, Q, AZ, AQ, gpu(st["beta"]), gpu(st["Pnext"][0]))
    col_close(host(Q)[:, :A.n], nx["Q"], 1e-13)
    col_close(host(AQ)[:, :A.n], nx["AQ"], 1e-13)
    gram_close(host(W), nx["W"], nx["Q"], nx["AQ"])
    gram_close(host(b1)[:, None], nx["b1"][:, None], nx["Q"], nx["r"][None, :])


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("k", [0, 3, 10])
def test_fgs_on_oracle_systems(traced, key, k):
    _, _, states, _ = traced[key]
    st = states[k]
    for sweeps in (1, 2, 3, 30):
        a, code = P.fgs(gpu(st["W"]), gpu(st["b1"]), sweeps)
        ar, _ = oracle.fgs(st["W"], st["b1"], sweeps)
        assert code == 0
        assert np.abs(host(a) - ar).max() <= 1e-12 * np.abs(ar).max()
        B, code = P.fgs(gpu(st["W"]), gpu(st["B2"]), sweeps)
        Br, _ = oracle.fgs(st["W"], st["B2"], sweeps)
        assert np.abs(host(B) - Br).max() <= 1e-12 * np.abs(Br).max()
    a, code = P.fgs(gpu(st["W"]), gpu(st["b1"]), 1, solver="cholesky")
    ar, _ = oracle.chol_solve(st["W"], st["b1"])
    # an exact solve: the difference is rounding times the condition of W
    assert np.abs(host(a) - ar).max() <= 1e-12 * np.linalg.cond(st["W"]) * np.abs(ar).max()


def test_fgs_status_flags():
    W = np.eye(4)
    W[2, 2] = 0.0
    _, code = P.fgs(gpu(W), gpu(np.ones(4)), 2)
    assert code == P.ERR_BREAKDOWN
    _, code = P.fgs(gpu(np.eye(4)), gpu(np.array([1.0, np.nan, 0, 0])), 2)
    assert code == P.ERR_NONFINITE
    _, code = P.fgs(gpu(-np.eye(3)), gpu(np.ones(3)), 1, solver="cholesky")
    assert code == P.ERR_BREAKDOWN


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("k", [0, 4])
def test_xr_update(traced, key, k):
    A, _, states, M = traced[key]
    st, nx = states[k], states[k + 1]
    ld = P.leading_dim(A.n)
    x, r = gpu(st["x"]), gpu(st["r"])
    z1 = torch.empty_like(x)
    rr = P.xr_update(M, block(st["Q"], ld), block(st["AQ"], ld), gpu(st["alpha"]), x, r, z1)
    col_close(host(x), nx["x"], 1e-13)
    col_close(host(r), nx["r"], 1e-13)
    col_close(host(z1), st["Znext"][0], 1e-13)
    assert abs(rr - oracle.dot(nx["r"], nx["r"])) <= 1e-12 * rr


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_xr_update_row_groups_match_single_rows(dtype):
    """16-byte aligned columns take R rows per thread, others one row per
    thread; every row's x, r and z1 are the same either way (only the sum
    order of ||r||^2 differs)."""
    A, _, _ = system("d27_17")   # n = 4913: a ragged tail for R = 2 and 4
    M = P.Matrix.from_csr(A, fp32=True, device=DEV)
    s, n = 6, A.n
    ld = P.leading_dim(n)
    rng = np.random.default_rng(12)
    Q = gpu(rng.normal(size=(s, ld)), dtype)
    AQ = gpu(rng.normal(size=(s, ld)), dtype)
    alpha = gpu(rng.normal(size=s))
    x0, r0 = rng.normal(size=n), rng.normal(size=n)
    out = []
    for offset in (0, 1):   # offset 1: x, r, z1 not 16-byte aligned
        vecs = []
        for v in (x0, r0, np.zeros(n)):
            buf = torch.zeros(n + offset, dtype=dtype, device=DEV)
            buf[offset:] = gpu(v, dtype)
            vecs.append(buf[offset:])
        rr = P.xr_update(M, Q, AQ, alpha, *vecs)
        out.append([host(v) for v in vecs] + [rr])
    for a, b in zip(out[0][:3], out[1][:3]):
        assert np.array_equal(a, b)
    assert abs(out[0][3] - out[1][3]) <= 1e-13 * out[1][3]
    xr = x0 + host(Q)[:, :n].astype(float).T @ host(alpha)
    assert np.abs(out[0][0] - xr).max() <= (1e-13 if dtype == torch.float64 else 1e-6) * np.abs(xr).max()


@pytest.mark.parametrize("key", KEYS)
@pytest.mark.parametrize("k", [0, 2, 7])
def test_one_outer_iteration(traced, key, k):
    """Step-level teacher forcing: one GPU outer iteration from oracle state k."""
    A, interval, states, M = traced[key]
    st, nx = states[k], states[k + 1]
    s = st["Q"].shape[0]
    ld = P.leading_dim(A.n)
    x, r = gpu(st["x"]), gpu(st["r"])
    Q, AQ = block(st["Q"], ld), block(st["AQ"], ld)
    P.xr_update(M, Q, AQ, gpu(st["alpha"]), x, r)
    Z, Pm = P.mpk(M, r, s, interval, ld=ld)
    B2 = P.gram_rect(A.n, Q, Pm[1:])
    beta, code = P.fgs(gpu(st["W"]), B2, 2)
    assert code == 0
    W, b1 = P.block_update_gram(A.n, Z, Q, Pm[1:], AQ, beta, Pm[0])
    alpha, code = P.fgs(W, b1, 2)
    # T2: 1e-12 (measured <= 2.7e-14 on x, r, Q, AQ; 1.7e-15 on W in the
    # forward-error scale of its dot products; 9e-16 on alpha)
    col_close(host(x), nx["x"], 1e-12)
    col_close(host(r), nx["r"], 1e-12)
    col_close(host(Q)[:, :A.n], nx["Q"], 1e-12)
    col_close(host(AQ)[:, :A.n], nx["AQ"], 1e-12)
    gram_close(host(W), nx["W"], nx["Q"], nx["AQ"], tol=1e-12)
    assert np.abs(host(alpha) - nx["alpha"]).max() <= 1e-12 * np.abs(nx["alpha"]).max()


def test_fp32_gram_kernels_match_upcast_oracle():
    A, _, interval = system("d7_13")
    s = 4
    rng = np.random.default_rng(9)
    Z = rng.normal(size=(s, A.n)).astype(np.float32)
    AZ = rng.normal(size=(s, A.n)).astype(np.float32)
    Q = rng.normal(size=(s, A.n)).astype(np.float32)
    AQ = rng.normal(size=(s, A.n)).astype(np.float32)
    r = rng.normal(size=A.n).astype(np.float32)
    beta = rng.normal(size=(s, s)) * 0.3
    B2 = P.gram_rect(A.n, gpu(Q), gpu(AZ))
    gram_close(host(B2), oracle.gram_rect(Q, AZ), Q.astype(float), AZ.astype(float))
    Qo, AQo = Q.copy(), AQ.copy()
    oracle.block_update(Z, Qo, AZ, AQo, beta)
    Qg, AQg = gpu(Q), gpu(AQ)
    W, b1 = P.block_update_gram(A.n, gpu(Z), Qg, gpu(AZ), AQg, gpu(beta), gpu(r))
    # each element is one FP32 rounding of nearly the same FP64 value
    d = np.abs(host(Qg).astype(np.float64) - Qo.astype(np.float64))
    assert np.all(d <= np.spacing(np.abs(Qo)).astype(np.float64) * 1.0001)
    Wr, br = oracle.gram(host(Qg), host(AQg), r)
    gram_close(host(W), Wr, host(Qg).astype(float), host(AQg).astype(float))



@pytest.mark.parametrize("n,ld,offset", [
    (2197, 2240, 0),     # 4 rows per thread, ragged tail of 1 row
    (4098, 4160, 0),     # tail of 2 rows
    (70001, 70016, 0),   # many 1024-row tiles and a tail
    (4099, 4099, 0),     # ld not a multiple of 4: one row per thread
    (4096, 4096, 1),     # columns not 16-byte aligned: one row per thread
])
def test_fp32_gram_rect_row_groups(n, ld, offset):
    s = 5
    rng = np.random.default_rng(n + offset)
    Q = rng.normal(size=(s, n)).astype(np.float32)
    AZ = rng.normal(size=(s, n)).astype(np.float32)

    def on_device(X):
        buf = torch.full((offset + s * ld,), float("nan"), dtype=torch.float32, device=DEV)
        view = buf[offset:].view(s, ld)
        view[:, :n] = gpu(X)
        return view

    B2 = P.gram_rect(n, on_device(Q), on_device(AZ))
    gram_close(host(B2), oracle.gram_rect(Q, AZ), Q.astype(float), AZ.astype(float))

# ------------------------------------------------------------- differentiation
def test_diffusion_kernels_match_oracle():
    N = 9
    theta = si.theta_field(N**3)
    A = si.stencil("7pt", N, np.exp(theta))
    M = P.Matrix.from_csr(A, device=DEV)
    val = host(P.diffusion7_assemble(M, gpu(theta)))
    ref = oracle.diffusion7_assemble(A, theta)
    assert np.abs(val - ref).max() <= 1e-14 * np.abs(ref).max()
    rng = np.random.default_rng(10)
    lam, x = rng.normal(size=A.n), rng.normal(size=A.n)
    g = host(P.csr_value_grad(M, gpu(lam), gpu(x)))
    assert np.array_equal(g, oracle.csr_value_grad(A, lam, x))
    gt = host(P.diffusion7_theta_grad(M, gpu(theta), gpu(g)))
    gr = oracle.diffusion7_theta_grad(A, theta, g)
    assert np.abs(gt - gr).max() <= 1e-12 * np.abs(gr).max()


def test_matrix_create_rejects_bad_input():
    A = si.poisson5(8)
    bad = A.val.copy()
    bad[A.row_ptr[3]] *= 1.0
    d = A.col == np.repeat(np.arange(A.n), np.diff(A.row_ptr))
    neg = A.val.copy()
    neg[np.flatnonzero(d)[5]] *= -1
    with pytest.raises(P.SSPCGError) as e:
        P.Matrix(A.row_ptr, A.col, neg, device=DEV)
    assert e.value.status == P.ERR_BREAKDOWN
    col = A.col.copy()
    col[7] = A.n + 3
    with pytest.raises(P.SSPCGError) as e:
        P.Matrix(A.row_ptr, col, A.val, device=DEV)
    assert e.value.status == P.ERR_ARG
    nanv = A.val.copy()
    nanv[2] = np.nan
    with pytest.raises(P.SSPCGError) as e:
        P.Matrix(A.row_ptr, A.col, nanv, device=DEV)
    assert e.value.status == P.ERR_NONFINITE


def random_spd_csr(n=1500, per_row=9, seed=21, unsorted=False):
    """Symmetric, strictly diagonally dominant matrix with a random pattern
    (its slices need explicit column indices)."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(n), per_row)
    cols = rng.integers(0, n, size=n * per_row)
    vals = -rng.uniform(0.1, 1.0, size=n * per_row)
    M = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    M = M + M.T
    M.setdiag(0.0)
    M.eliminate_zeros()
    d = np.asarray(abs(M).sum(axis=1)).ravel() + rng.uniform(0.5, 2.0, n)
    M = (M + sp.diags(d)).tocsr()
    M.sort_indices()
    rp, col, val = M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.copy()
    if unsorted:
        for i in range(n):
            a, b = rp[i], rp[i + 1]
            perm = rng.permutation(b - a)
            col[a:b] = col[a:b][perm]
            val[a:b] = val[a:b][perm]
    return si.CSR(n, rp, col, val, (1, 1, n))


@pytest.mark.parametrize("unsorted", [False, True])
def test_explicit_column_slices(unsorted):
    A = random_spd_csr(unsorted=unsorted)
    M = P.Matrix.from_csr(A, fp32=True, device=DEV)
    assert M.info()["slots"] >= A.nnz
    x = np.random.default_rng(22).normal(size=A.n)
    y = host(P.spmv(M, gpu(x)))
    ref = oracle.spmv(A, x)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()
    x32 = x.astype(np.float32)
    assert np.array_equal(host(P.spmv(M, gpu(x32))),
                          oracle.spmv_f32(A, A.val.astype(np.float32), x32))
    b = si.rhs_uniform(A.n)
    dinv = oracle.jacobi_inverse(A)
    Dh = np.sqrt(dinv)
    ev = np.linalg.eigvalsh(si.to_scipy(A).toarray() * np.outer(Dh, Dh))
    x_g, info = P.solve(M, gpu(b), s=4, sweeps=3, interval=(ev[0], ev[-1]), tol=1e-12)
    x_o, ro = oracle.sspcg(A, b, s=4, sweeps=3, interval=(ev[0], ev[-1]), tol=1e-12)
    assert info["status"] == ro["status"] == 0
    assert np.linalg.norm(host(x_g) - x_o) <= 1e-10 * np.linalg.norm(x_o)


def test_stencil_slices_use_shared_offsets():
    """A stencil matrix stores one offset list per slice: slots ~ stencil size x rows."""
    N = 32
    A = si.stencil("27pt", N, si.coeff_blocks(N))
    M = P.Matrix.from_csr(A, device=DEV)
    info = M.info()
    # every slice shares one offset list: the 27 stencil offsets inside the
    # grid, fewer on boundary planes (slices hold 64 rows of one x-line half)
    assert info["shared_slices"] == info["slices"] == N**3 // 64
    # symmetric: the diagonal and the 13 upper offsets of every row
    assert info["symmetric"] == 1 and info["slots"] == 14 * N**3
    # values only: 8 bytes per slot plus small metadata, no column indices
    assert info["device_bytes"] < 8 * info["slots"] + 40 * A.n
    Mf = P.Matrix.from_csr(A, full_storage=True, device=DEV)
    assert Mf.info()["symmetric"] == 0 and A.nnz <= Mf.info()["slots"] <= 27 * N**3


@pytest.mark.parametrize("key", KEYS)
def test_fgs_sweep_tol_on_oracle_systems(traced, key):
    _, _, states, _ = traced[key]
    st = states[3]
    for d in (1e-1, 1e-4):
        a, code = P.fgs(gpu(st["W"]), gpu(st["b1"]), 300, sweep_tol=d)
        ar, _ = oracle.fgs(st["W"], st["b1"], 300, sweep_tol=d)
        assert code == 0
        assert np.abs(host(a) - ar).max() <= 1e-10 * np.abs(ar).max()
        B, code = P.fgs(gpu(st["W"]), gpu(st["B2"]), 300, sweep_tol=d)
        Br, _ = oracle.fgs(st["W"], st["B2"], 300, sweep_tol=d)
        assert np.abs(host(B) - Br).max() <= 1e-10 * np.abs(Br).max()


@pytest.mark.parametrize("s", [2, 6])
def test_mpk_monomial(sys_, s):
    A, _, interval, M = sys_
    dinv = oracle.jacobi_inverse(A)
    r = np.random.default_rng(41).uniform(-1, 1, A.n)
    Zr, Pr = oracle.mpk(A, dinv, r, s, interval, basis="monomial")
    Z, Pm = P.mpk(M, gpu(r), s, interval, basis="monomial")
    col_close(host(Z), Zr, 1e-12)
    col_close(host(Pm), Pr, 1e-12)


# ---------------------------------------------------------------- basis interval estimates
# Lanczos: the tridiagonal coefficients follow the oracle's to rounding, and
# 20 steps amplify those differences only mildly, so the Ritz values agree to
# 1e-9 relative.  Power method: every step is a normalised SpMV, 1e-12.


def test_interval_lanczos_matches_oracle(sys_):
    A, _, _, M = sys_
    v0 = si.start_vector(A.n)
    out = P.interval(M, gpu(v0), method="lanczos", steps=20)
    lo, hi, k = oracle.lanczos_bounds(A, v0, 20)
    assert out["steps"] == k == 20
    glo, ghi = out["interval"]
    assert abs(glo - lo) <= 1e-9 * abs(lo) and abs(ghi - hi) <= 1e-9 * abs(hi)


def test_interval_power_matches_oracle(sys_):
    A, _, _, M = sys_
    v0 = si.start_vector(A.n)
    for rtol, steps in ((1e-3, 50), (0.0, 30)):
        out = P.interval(M, gpu(v0), method="power", steps=steps, rtol=rtol)
        lo, hi, k, hist = oracle.power_bounds(A, v0, rtol=rtol, max_iter=steps)
        assert out["interval"][0] == 0.0
        rel = np.abs(np.diff(hist)) / hist[1:]
        # the stop step is an integer decided in FP64; compare it exactly
        # unless the oracle's decision was within rounding of rtol
        if np.all(np.abs(rel - rtol) > 1e-9 * max(rtol, 1e-300)):
            assert out["steps"] == k
            assert abs(out["interval"][1] - hi) <= 1e-12 * hi
        else:
            assert abs(out["steps"] - k) <= 1


def test_interval_lanczos_full_run_and_step_cap():
    # steps > n: capped at n; the extremes are then the closed-form ones
    N = 8
    A = si.poisson5(N)
    M = P.Matrix.from_csr(A, device=DEV)
    out = P.interval(M, gpu(si.start_vector(A.n)), method="lanczos", steps=100)
    clo, chi = si.closed_form_bounds("5pt", N)
    assert out["steps"] == A.n
    assert abs(out["interval"][0] - clo) <= 1e-12 and abs(out["interval"][1] - chi) <= 1e-12


def test_interval_lanczos_invariant_start_stops_after_one_step():
    n = 40
    d = 4.0 ** np.arange(-5, n - 5)
    A = si.CSR(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), d, None)
    M = P.Matrix.from_csr(A, device=DEV)
    v0 = np.zeros(n)
    v0[7] = 3.0
    out = P.interval(M, gpu(v0), method="lanczos", steps=20)
    assert out == {"interval": (1.0, 1.0), "steps": 1}
    assert oracle.lanczos_bounds(A, v0, 20) == (1.0, 1.0, 1)


def test_interval_rejects_bad_input():
    A = si.poisson5(16)
    M = P.Matrix.from_csr(A, device=DEV)
    with pytest.raises(P.SSPCGError) as e:
        P.interval(M, torch.zeros(A.n, dtype=torch.float64, device=DEV))
    assert e.value.status == P.ERR_ARG
    bad = si.start_vector(A.n)
    bad[3] = np.nan
    with pytest.raises(P.SSPCGError) as e:
        P.interval(M, gpu(bad), method="power")
    assert e.value.status == P.ERR_ARG
    for kw in (dict(steps=0), dict(steps=1001), dict(method="power", rtol=-1.0)):
        with pytest.raises(P.SSPCGError) as e:
            P.interval(M, gpu(si.start_vector(A.n)), **kw)
        assert e.value.status == P.ERR_ARG
    # the matrix still works afterwards
    out = P.interval(M, gpu(si.start_vector(A.n)), method="lanczos", steps=5)
    assert out["steps"] == 5



# ---------------------------------------------------------------- symmetric half storage


@pytest.mark.parametrize("kind,N", [("5pt", 40), ("7pt", 13), ("27pt", 17)])
def test_half_storage_is_the_same_product(kind, N):
    """One triangle stored: the SpMV sums the same terms in the same order, so
    FP64 and FP32 products equal the full storage's bit for bit."""
    n = N * N if kind == "5pt" else N**3
    kap = np.exp(si.theta_field(n))
    A = si.stencil(kind, N, kap)
    Mh = P.Matrix.from_csr(A, fp32=True, device=DEV)
    Mf = P.Matrix.from_csr(A, fp32=True, full_storage=True, device=DEV)
    assert Mh.info()["symmetric"] == 1 and Mf.info()["symmetric"] == 0
    assert Mh.info()["device_bytes"] < 0.7 * Mf.info()["device_bytes"]
    rng = np.random.default_rng(40)
    x = gpu(rng.normal(size=A.n))
    assert torch.equal(P.spmv(Mh, x), P.spmv(Mf, x))
    x32 = x.float()
    assert torch.equal(P.spmv(Mh, x32), P.spmv(Mf, x32))
    interval = si.lanczos_bounds(A)
    for Z, Pm in zip(P.mpk(Mh, x, 6, interval), P.mpk(Mf, x, 6, interval)):
        assert torch.equal(Z, Pm)


def test_nonsymmetric_stencil_keeps_full_storage():
    N = 12
    A = si.stencil("7pt", N, np.exp(si.theta_field(N**3)))
    val = A.val.copy()
    val[A.row_ptr[100] + 1] *= 1.0 + 2.0**-40      # one off-diagonal entry, one ulp-ish off
    B = si.CSR(A.n, A.row_ptr, A.col, val, A.shape3)
    M = P.Matrix.from_csr(B, fp32=True, device=DEV)
    assert M.info()["symmetric"] == 0
    x = np.random.default_rng(41).normal(size=A.n)
    y = host(P.spmv(M, gpu(x)))
    ref = oracle.spmv(B, x)
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max()
    x32 = x.astype(np.float32)
    assert np.array_equal(host(P.spmv(M, gpu(x32))), oracle.spmv_f32(B, B.val.astype(np.float32), x32))


def test_update_values_checks_before_changing_anything():
    N = 12
    A = si.stencil("7pt", N, np.exp(si.theta_field(N**3)))
    M = P.Matrix.from_csr(A, device=DEV)
    assert M.info()["symmetric"] == 1
    x = gpu(np.random.default_rng(42).normal(size=A.n))
    interval = si.lanczos_bounds(A)
    y0 = P.spmv(M, x).clone()
    Z0, _ = P.mpk(M, x, 3, interval)            # uses 1/diag(A) too
    # not symmetric: refused on a half-storage matrix, nothing changed
    bad = A.val.copy()
    bad[A.row_ptr[50] + 1] *= 1.5
    with pytest.raises(P.SSPCGError) as e:
        M.update_values(gpu(bad))
    assert e.value.status == P.ERR_UNSUPPORTED
    # non-finite and non-positive diagonal: refused, nothing changed
    nan = A.val.copy()
    nan[7] = np.nan
    with pytest.raises(P.SSPCGError) as e:
        M.update_values(gpu(nan))
    assert e.value.status == P.ERR_NONFINITE
    neg = A.val.copy()
    diag = [a for i in range(A.n) for a in range(A.row_ptr[i], A.row_ptr[i + 1]) if A.col[a] == i]
    neg[diag[3]] = -1.0
    with pytest.raises(P.SSPCGError) as e:
        M.update_values(gpu(neg))
    assert e.value.status == P.ERR_BREAKDOWN
    assert torch.equal(P.spmv(M, x), y0)
    assert torch.equal(P.mpk(M, x, 3, interval)[0], Z0)
    # symmetric new values are accepted and used
    M.update_values(gpu(2.0 * A.val))
    assert torch.equal(P.spmv(M, x), 2.0 * y0)
    # full storage accepts non-symmetric values
    Mf = P.Matrix.from_csr(A, full_storage=True, device=DEV)
    Mf.update_values(gpu(bad))
    Bm = si.CSR(A.n, A.row_ptr, A.col, bad, A.shape3)
    ref = oracle.spmv(Bm, host(x))
    assert np.abs(host(P.spmv(Mf, x)) - ref).max() <= 1e-14 * np.abs(ref).max()


def stencil_csr(kind, N):
    """9-point 2D (list length 9) or 19-point 3D (19) stencils: no
    compile-time row variant exists for them, so the generic ones run."""
    import scipy.sparse as sp
    B = sp.diags([1.0, 1.0, 1.0], [-1, 0, 1], shape=(N, N))
    if kind == "9pt":
        K = sp.kron(B, B)                       # centre + 8 neighbours
        A = 9.5 * sp.eye(N * N) - K
        shape = (1, N, N)
    else:
        # 19 points: the 3x3x3 cube without its 8 corners
        I = sp.eye(N)
        T = sp.diags([1.0, 1.0], [-1, 1], shape=(N, N))
        faces = sp.kron(sp.kron(T, I), I) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(I, I), T)
        edges = sp.kron(sp.kron(T, T), I) + sp.kron(sp.kron(T, I), T) + sp.kron(sp.kron(I, T), T)
        A = 19.5 * sp.eye(N**3) - faces - 0.5 * edges
        shape = (N, N, N)
    A = A.tocsr()
    A.sort_indices()
    rng = np.random.default_rng(44)
    # symmetric positive scaling keeps A symmetric and varies the values
    d = rng.uniform(0.5, 2.0, A.shape[0])
    A = (sp.diags(d) @ A @ sp.diags(d)).tocsr()
    A.sort_indices()
    return si.CSR(A.shape[0], A.indptr.astype(np.int32), A.indices.astype(np.int32),
                  A.data.copy(), shape)


@pytest.mark.parametrize("kind,N", [("9pt", 48), ("9pt", 37), ("19pt", 12), ("19pt", 9)])
@pytest.mark.parametrize("full", [False, True])
def test_generic_stencil_rows(kind, N, full):
    A = stencil_csr(kind, N)
    M = P.Matrix.from_csr(A, fp32=True, full_storage=full, device=DEV)
    info = M.info()
    assert info["symmetric"] == (0 if full else 1)
    x = np.random.default_rng(45).normal(size=A.n)
    y = host(P.spmv(M, gpu(x)))
    ref = oracle.spmv(A, x)
    absA = A.__class__(A.n, A.row_ptr, A.col, np.abs(A.val), A.shape3)
    assert np.all(np.abs(y - ref) <= 1e-14 * oracle.spmv(absA, np.abs(x)))
    x32 = x.astype(np.float32)
    assert np.array_equal(host(P.spmv(M, gpu(x32))), oracle.spmv_f32(A, A.val.astype(np.float32), x32))
    b = si.rhs_uniform(A.n)
    interval = si.lanczos_bounds(A)
    xg, ig = P.solve(M, gpu(b), s=4, sweeps=3, interval=interval, tol=1e-30, max_outer=15)
    xo, ro = oracle.sspcg(A, b, s=4, sweeps=3, interval=interval, tol=1e-30, max_outer=15)
    assert ig["outer_iters"] == ro["iters"] == 15
    assert np.linalg.norm(host(xg) - xo) <= 1e-10 * np.linalg.norm(xo)


def banded_csr(n, offsets, seed):
    """Symmetric, diagonally dominant matrix whose rows all use the offsets
    +-o (o in offsets) and 0: a uniform layout whose offset list has one
    run of consecutive values per isolated offset."""
    import scipy.sparse as sp
    rng = np.random.default_rng(seed)
    diags, offs = [], []
    for o in offsets:
        v = rng.uniform(-1.0, -0.1, n - o)
        diags += [v, v]
        offs += [o, -o]
    M = sp.diags(diags, offs, shape=(n, n)).tocsr()
    d = np.asarray(abs(M).sum(axis=1)).ravel() + 1.0
    M = (M + sp.diags(d)).tocsr()
    M.sort_indices()
    return si.CSR(n, M.indptr.astype(np.int32), M.indices.astype(np.int32), M.data.copy(),
                  (1, 1, n))


@pytest.mark.parametrize("nruns", [11, 13])
@pytest.mark.parametrize("spacing", ["near", "far"])
@pytest.mark.parametrize("full", [False, True])
def test_many_offset_runs(nruns, spacing, full):
    """2k+1 isolated offsets (a mirrored list always has an odd number of
    runs).  Near offsets (less than a tile apart) share one LDS window of x;
    far ones (more than a tile apart) take a window each: up to 12 windows x
    is staged in LDS (FP64), beyond that the rows gather from memory.  Every
    case must give the oracle's product and iterates."""
    k = (nruns - 1) // 2
    if spacing == "near":
        offsets = [3 * (i + 1) + i * i for i in range(k)]        # no two consecutive
    else:
        offsets = [257 * (i + 1) + i for i in range(k)]          # gaps beyond a tile
    n = 64 * 37 + 11
    A = banded_csr(n, offsets, seed=46 + nruns)
    M = P.Matrix.from_csr(A, fp32=True, full_storage=full, device=DEV)
    assert M.info()["symmetric"] == (0 if full else 1)
    x = np.random.default_rng(47).normal(size=A.n)
    y = host(P.spmv(M, gpu(x)))
    ref = oracle.spmv(A, x)
    absA = A.__class__(A.n, A.row_ptr, A.col, np.abs(A.val), A.shape3)
    assert np.all(np.abs(y - ref) <= 1e-14 * oracle.spmv(absA, np.abs(x)))
    x32 = x.astype(np.float32)
    assert np.array_equal(host(P.spmv(M, gpu(x32))), oracle.spmv_f32(A, A.val.astype(np.float32), x32))
    b = si.rhs_uniform(A.n)
    interval = si.lanczos_bounds(A)
    xg, ig = P.solve(M, gpu(b), s=4, sweeps=3, interval=interval, tol=1e-30, max_outer=12)
    xo, ro = oracle.sspcg(A, b, s=4, sweeps=3, interval=interval, tol=1e-30, max_outer=12)
    assert ig["outer_iters"] == ro["iters"] == 12
    assert np.linalg.norm(host(xg) - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.parametrize("n", [4099, 4096])
def test_update_gram_row_groups_match_single_rows(n):
    """FP32 block update: with 16-byte aligned columns four rows per thread
    (the rows of a ragged tail one by one), otherwise one row per thread
    (ld not a multiple of 4).  Q and AQ are the same bits either way; W and
    b1 only sum the rows in another order."""
    s = 6
    rng = np.random.default_rng(31)
    beta = gpu(rng.normal(size=(s, s)) * 0.3)
    cols = [rng.normal(size=(s, n)).astype(np.float32) for _ in range(4)]
    r = rng.normal(size=n).astype(np.float32)
    out = []
    for ld in (P.leading_dim(n), n + 1 if n % 4 == 0 else n + 2):
        Z, Q, AZ, AQ = (torch.zeros((s, ld), dtype=torch.float32, device=DEV) for _ in range(4))
        for t, c in zip((Z, Q, AZ, AQ), cols):
            t[:, :n] = gpu(c)
        W, b1 = P.block_update_gram(n, Z, Q, AZ, AQ, beta, gpu(r))
        out.append((host(Q)[:, :n], host(AQ)[:, :n], host(W), host(b1)))
    (q0, aq0, w0, b0), (q1, aq1, w1, b1_) = out
    assert np.array_equal(q0, q1) and np.array_equal(aq0, aq1)
    Qd, AQd = q0.astype(float), aq0.astype(float)
    gram_close(w0, w1, Qd, AQd, tol=1e-13)
    gram_close(b0[:, None], b1_[:, None], Qd, r.astype(float)[None, :], tol=1e-13)
    Wr, br = oracle.gram(q0, aq0, r)
    gram_close(w0, Wr, Qd, AQd)


# ---------------------------------------------------------------- bandwidth reference


@pytest.mark.parametrize("n", [1, 7, 256 * 8 + 3, 1 << 20, (1 << 20) + 1])
def test_stream_triad(n):
    """a = b + q c, with q a power of two so that q c is exact and the FMA and
    the separate product and sum round alike: bit for bit against numpy, also
    for odd lengths (the last element in a kernel of its own) and lengths
    that leave a ragged last tile."""
    rng = np.random.default_rng(60 + n % 97)
    b, c = rng.normal(size=n), rng.normal(size=n)
    q = 0.125
    a = torch.full((n,), np.nan, dtype=torch.float64, device=DEV)
    P.stream_triad(a, gpu(b), gpu(c), q)
    assert np.array_equal(host(a), b + q * c)
