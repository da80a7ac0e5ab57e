"""Step-level parity of the HIP path with the oracle (each test calls the C ABI through the
binding, on seeded inputs, and compares with the oracle's plain definition of that step).
Sizes span several GEMM/LU tiles with ragged tails."""
import numpy as np
import pytest

import workloads as wl
from oracle import dense, quadrature as qd

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1801_09794_amd as nl  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def gpu():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    nl.lib()      # raises if the library is not built
    yield
    torch.cuda.synchronize()


def dev(A, dtype=torch.complex128):
    return nl.to_colmajor(A, "cuda", dtype)


def batch_dev(mats, dtype=torch.complex128):
    return torch.stack([dev(M, dtype) for M in mats])


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)

def solve_tol(dtype, M):
    """Bound on the relative error of a solve with the LU factors of M: the normwise forward
    error of a backward-stable solve is about g * cond(M) * u; g = 20 leaves room for the
    complex64 factors, whose products take the 3M scheme (imaginary parts rounded up to about
    twice as coarsely as with four real products).  complex128 keeps the fixed 1e-11."""
    if dtype == "c128":
        return 1e-11
    return 20 * np.linalg.cond(M) * 2.0 ** -24



@pytest.mark.parametrize("dt,tol", [(torch.complex128, 1e-14), (torch.complex64, 3e-6)])
def test_mfma_lane_layout_single_tile(dt, tol):
    # one 16x16x4 block per dtype: catches a wrong MFMA operand/accumulator lane layout
    rng = np.random.default_rng(0)
    if True:
        A = wl.cn(rng, (16, 4))
        B = wl.cn(rng, (4, 16))
        C = torch.zeros((16, 16), dtype=dt, device="cuda")
        nl.nlf_gemm_batched("N", 16, 16, 4, 1.0, dev(A, dt), 16, 0, dev(B, dt), 4, 0, 0.0, C, 16, 0, 1)
        torch.cuda.synchronize()
        assert rel(nl.from_colmajor(C), A @ B) < tol


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("opA", ["N", "C"])
@pytest.mark.parametrize("M,N,K,batch", [(37, 53, 29, 1), (130, 70, 300, 3), (257, 129, 64, 2),
                                         (64, 64, 3000, 2), (1, 1, 1, 1), (200, 5, 0, 1)])
def test_gemm_matches_definition(dtype, opA, M, N, K, batch):
    rng = np.random.default_rng(M * 7 + N + K)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-13 if dtype == "c128" else 2e-5
    As = [wl.cn(rng, (M, K) if opA == "N" else (K, M)) for _ in range(batch)]
    Bs = [wl.cn(rng, (K, N)) for _ in range(batch)]
    Cs = [wl.cn(rng, (M, N)) for _ in range(batch)]
    alpha, beta = 0.7 - 0.2j, -0.3 + 1.1j
    Ad, Bd, Cd = batch_dev(As, dt), batch_dev(Bs, dt), batch_dev(Cs, dt)
    lda = M if opA == "N" else K
    nl.nlf_gemm_batched(opA, M, N, K, alpha, Ad, max(lda, 1), As[0].size, Bd, max(K, 1), Bs[0].size,
                        beta, Cd, M, Cs[0].size, batch)
    torch.cuda.synchronize()
    for b in range(batch):
        opa = As[b] if opA == "N" else As[b].conj().T
        ref = alpha * (opa @ Bs[b]) + beta * Cs[b]
        got = nl.from_colmajor(Cd[b])
        assert rel(got, ref) < tol * max(1, np.sqrt(K))


def test_assemble_matches_oracle():
    rng = np.random.default_rng(1)
    n = 300
    terms = wl.DELAY
    mats = [wl.cn(rng, (n, n)) for _ in terms]
    C = qd.Contour(0.2 + 0.5j, 0.3)
    z, _ = qd.nodes_weights(C, 5)
    T64 = torch.empty((5, n, n), dtype=torch.complex128, device="cuda")
    T32 = torch.empty((5, n, n), dtype=torch.complex64, device="cuda")
    nl.nlf_assemble(terms, [dev(M) for M in mats], z, T64, T32)
    torch.cuda.synchronize()
    ref = dense.assemble(terms, mats, z)
    for k in range(5):
        assert rel(nl.from_colmajor(T64[k]), ref[k]) < 1e-15
        r32 = ref[k].astype(np.complex64)
        assert np.array_equal(nl.from_colmajor(T32[k]), r32) or rel(nl.from_colmajor(T32[k]), ref[k]) < 1e-7


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("M,N,K,batch,odd_ld", [(2048, 1536, 80, 2, False), (1024, 2048, 512, 2, False),
                                                (2048, 1536, 80, 2, True), (2000, 1530, 96, 2, False),
                                                (2046, 1500, 64, 2, False), (2047, 1530, 96, 2, False),
                                                (2048, 1536, 88, 2, False), (2048, 1568, 80, 2, False)])
def test_gemm_direct_lds_tile_matches_definition(dtype, M, N, K, batch, odd_ld):
    # products with op(A) = A that fill the chip with 64 x 64 (complex128) or 128 x 64 (complex64)
    # tiles: the direct-to-LDS 3M forms, here on sub-matrices (leading dimensions above the row
    # counts) with general alpha and beta.  Full tiles; ragged rows and columns (predicated loads,
    # idle waves, guarded stores; complex128 with at most 32 ragged columns splits them off onto
    # 64 x 32 tiles, full for N = 1568 = 24 x 64 + 32, ragged for N = 1500); an
    # odd leading dimension or an odd row count (complex64 element pairs lose their 16-byte
    # alignment) and a reduction that is not a multiple of 16 take the staged form
    rng = np.random.default_rng(M + 3 * N + K + odd_ld)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-13 if dtype == "c128" else 2e-5
    lda, ldb, ldc = M + 64 + odd_ld, K + 16 + odd_ld, M + 128
    alpha, beta = -1.0 + 0.25j, 0.5 - 0.75j
    A = [wl.cn(rng, (lda, K)) for _ in range(batch)]
    B = [wl.cn(rng, (ldb, N)) for _ in range(batch)]
    C = [wl.cn(rng, (ldc, N)) for _ in range(batch)]
    if dtype == "c64":
        A, B, C = ([X.astype(np.complex64).astype(complex) for X in Y] for Y in (A, B, C))
    Ad, Bd, Cd = batch_dev(A, dt), batch_dev(B, dt), batch_dev(C, dt)
    nl.nlf_gemm_batched("N", M, N, K, alpha, Ad, lda, lda * K, Bd, ldb, ldb * N, beta, Cd, ldc, ldc * N, batch)
    torch.cuda.synchronize()
    for b in range(batch):
        got = nl.from_colmajor(Cd[b]).astype(complex)
        ref = C[b].copy()
        ref[:M] = alpha * (A[b][:M] @ B[b][:K]) + beta * C[b][:M]
        assert rel(got[:M], ref[:M]) < tol * np.sqrt(K)
        assert np.array_equal(got[M:], C[b][M:])      # rows between M and ldc untouched


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,batch", [(1, 2), (7, 3), (33, 2), (100, 2), (257, 2), (600, 1)])
def test_getrf_matches_oracle_lu(dtype, n, batch):
    rng = np.random.default_rng(n + batch)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    mats = [wl.cn(rng, (n, n)) for _ in range(batch)]
    if dtype == "c64":
        mats = [M.astype(np.complex64).astype(complex) for M in mats]
    A = batch_dev(mats, dt)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    nl.nlf_getrf_batched(A, ipiv, perm, info)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0] * batch
    for b in range(batch):
        LU = nl.from_colmajor(A[b]).astype(complex)
        piv = ipiv[b].cpu().numpy()
        L = np.tril(LU, -1) + np.eye(n)
        U = np.triu(LU)
        PA = dense.apply_pivots(piv, mats[b])
        eps = 2.2e-16 if dtype == "c128" else 1.2e-7
        assert np.max(np.abs(PA - L @ U)) <= 30 * n * eps * np.max(np.abs(mats[b]))
        assert np.all(piv >= np.arange(n)) and np.all(piv < n)
        p = perm[b].cpu().numpy()
        assert np.array_equal(np.sort(p), np.arange(n))
        assert np.array_equal(mats[b][p], PA)
        if dtype == "c128" and n <= 257:
            LU0, piv0 = dense.lu_partial_pivot(mats[b])
            assert np.array_equal(piv, piv0)
            assert rel(LU, LU0) < 1e-12


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,batch", [(33, 2), (256, 2), (300, 2), (700, 2), (1100, 1)])
def test_getrf_blocked_matches_oracle_and_inverses(dtype, n, batch):
    # right-looking blocked LU with 512-column panels: one partial panel (one or two inverse
    # blocks), a ragged second panel, three panels with a ragged third; the 256 x 256
    # diagonal-block inverses it leaves behind are checked as well
    rng = np.random.default_rng(7 * n + batch)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    mats = [wl.cn(rng, (n, n)) for _ in range(batch)]
    if dtype == "c64":
        mats = [M.astype(np.complex64).astype(complex) for M in mats]
    A = batch_dev(mats, dt)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    per = nl.nlf_lu_inverse_elems(n)
    dinv = torch.empty(batch * per, dtype=dt, device="cuda")
    nl.nlf_getrf_batched_blocked(A, ipiv, perm, info, dinv)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0] * batch
    eps = 2.2e-16 if dtype == "c128" else 1.2e-7
    D = dinv.cpu().numpy().astype(complex)
    for b in range(batch):
        LU = nl.from_colmajor(A[b]).astype(complex)
        piv = ipiv[b].cpu().numpy()
        L = np.tril(LU, -1) + np.eye(n)
        U = np.triu(LU)
        assert np.max(np.abs(dense.apply_pivots(piv, mats[b]) - L @ U)) <= 30 * n * eps * np.max(np.abs(mats[b]))
        assert np.array_equal(mats[b][perm[b].cpu().numpy()], dense.apply_pivots(piv, mats[b]))
        if dtype == "c128":
            LU0, piv0 = dense.lu_partial_pivot(mats[b])
            assert np.array_equal(piv, piv0)
            assert rel(LU, LU0) < 1e-11
        for q in range(-(-n // 256)):
            s0, sb = 256 * q, min(256, n - 256 * q)
            blk = D[b * per + 2 * q * 65536: b * per + (2 * q + 2) * 65536]
            Li = blk[:65536].reshape(256, 256).T[:sb, :sb]
            Ui = blk[65536:].reshape(256, 256).T[:sb, :sb]
            tol = 1e-10 if dtype == "c128" else 1e-3
            assert np.max(np.abs(Li @ L[s0:s0 + sb, s0:s0 + sb] - np.eye(sb))) < tol
            assert np.max(np.abs(Ui @ U[s0:s0 + sb, s0:s0 + sb] - np.eye(sb))) < tol


def test_getrf_zero_pivot_info():
    A = np.eye(40, dtype=complex)
    A[17, 17] = 0.0
    A[:, 17] = 0.0
    d = batch_dev([A, np.eye(40, dtype=complex)])
    ipiv = torch.empty((2, 40), dtype=torch.int32, device="cuda")
    info = torch.empty(2, dtype=torch.int32, device="cuda")
    nl.nlf_getrf_batched(d, ipiv, None, info)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [18, 0]


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,nrhs,batch", [(100, 7, 2), (300, 64, 3), (1000, 20, 2)])
def test_getrs_matches_solve(dtype, n, nrhs, batch):
    rng = np.random.default_rng(n + nrhs)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    mats = [wl.cn(rng, (n, n)) + 3 * np.eye(n) for _ in range(batch)]
    B = wl.cn(rng, (n, nrhs))
    A = batch_dev(mats, dt)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    nl.nlf_getrf_batched(A, ipiv, perm, info)
    X = torch.empty((batch, nrhs, n), dtype=dt, device="cuda")
    nl.nlf_getrs_batched(A, perm, dev(B, dt), X, shared_rhs=True)
    torch.cuda.synchronize()
    for b in range(batch):
        ref = np.linalg.solve(mats[b], B)
        assert rel(nl.from_colmajor(X[b]), ref) < solve_tol(dtype, mats[b])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,nrhs,batch", [(100, 7, 2), (300, 64, 3), (700, 20, 2), (1000, 33, 1),
                                           (1200, 24, 2)])
def test_getrs_block_inverse_matches_solve(dtype, n, nrhs, batch):
    # n spans one partial 256-block, several blocks and a ragged last block; the updates outside
    # a chunk of four blocks come once per chunk (1200: five blocks, chunks of 4 and 1)
    rng = np.random.default_rng(n + 3 * nrhs)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    mats = [wl.cn(rng, (n, n)) + 3 * np.eye(n) for _ in range(batch)]
    B = wl.cn(rng, (n, nrhs))
    A = batch_dev(mats, dt)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    nl.nlf_getrf_batched(A, ipiv, perm, info)
    dinv = torch.empty(batch * nl.nlf_lu_inverse_elems(n), dtype=dt, device="cuda")
    nl.nlf_lu_block_inverses(A, dinv)
    X = torch.empty((batch, nrhs, n), dtype=dt, device="cuda")
    tmp = torch.empty(batch * 256 * nrhs, dtype=dt, device="cuda")
    nl.nlf_getrs_batched_inv(A, perm, dinv, dev(B, dt), X, tmp, shared_rhs=True)
    torch.cuda.synchronize()
    for b in range(batch):
        ref = np.linalg.solve(mats[b], B)
        assert rel(nl.from_colmajor(X[b]), ref) < solve_tol(dtype, mats[b])


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("n,nrhs,batch,inplace", [(100, 7, 2, False), (300, 64, 3, True), (700, 20, 2, False),
                                                  (1000, 33, 1, True), (1200, 24, 2, False)])
def test_getrs_adjoint_matches_solve(dtype, n, nrhs, batch, inplace):
    # X = A^{-H} B from the factors of A (the adjoint problem's solves): B shared by the batch
    # with a separate scratch Z, or one B per matrix used as Z itself
    rng = np.random.default_rng(n + 5 * nrhs)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    mats = [wl.cn(rng, (n, n)) + 3 * np.eye(n) for _ in range(batch)]
    Bs = [wl.cn(rng, (n, nrhs)) for _ in range(batch)]
    A = batch_dev(mats, dt)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    nl.nlf_getrf_batched(A, ipiv, perm, info)
    dinv = torch.empty(batch * nl.nlf_lu_inverse_elems(n), dtype=dt, device="cuda")
    nl.nlf_lu_block_inverses(A, dinv)
    X = torch.empty((batch, nrhs, n), dtype=dt, device="cuda")
    tmp = torch.empty(batch * 256 * nrhs, dtype=dt, device="cuda")
    if inplace:
        B = torch.stack([dev(b, dt) for b in Bs])
        nl.nlf_getrs_batched_inv_adjoint(A, perm, dinv, B, B, X, tmp)
        refs = [np.linalg.solve(M.conj().T, b) for M, b in zip(mats, Bs)]
    else:
        Z = torch.empty((batch, nrhs, n), dtype=dt, device="cuda")
        nl.nlf_getrs_batched_inv_adjoint(A, perm, dinv, dev(Bs[0], dt), Z, X, tmp, shared_rhs=True)
        refs = [np.linalg.solve(M.conj().T, Bs[0]) for M in mats]
    torch.cuda.synchronize()
    for b in range(batch):
        assert rel(nl.from_colmajor(X[b]), refs[b]) < solve_tol(dtype, mats[b])


def test_getrs_adjoint_rejects_overlap():
    n, nrhs = 64, 4
    A = torch.zeros((1, n, n), dtype=torch.complex128, device="cuda")
    perm = torch.zeros((1, n), dtype=torch.int32, device="cuda")
    dinv = torch.zeros(nl.nlf_lu_inverse_elems(n), dtype=torch.complex128, device="cuda")
    Z = torch.zeros((1, nrhs, n), dtype=torch.complex128, device="cuda")
    tmp = torch.zeros(256 * nrhs, dtype=torch.complex128, device="cuda")
    with pytest.raises(nl.NLFError) as e:
        nl.nlf_getrs_batched_inv_adjoint(A, perm, dinv, Z, Z, Z, tmp)
    assert e.value.status == nl.NLF_ERR_ARG


def test_getrf_large_backward_error():
    # n = 4096: several recursion levels, 4 rows per panel thread, full-size panels
    n, batch = 4096, 2
    rng = np.random.default_rng(44)
    mats = [wl.cn(rng, (n, n)) / np.sqrt(n) for _ in range(batch)]
    A = batch_dev(mats)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    nl.nlf_getrf_batched(A, ipiv, perm, info)
    B = wl.cn(rng, (n, 8))
    X = torch.empty((batch, 8, n), dtype=torch.complex128, device="cuda")
    nl.nlf_getrs_batched(A, perm, dev(B), X, shared_rhs=True)
    dinv = torch.empty(batch * nl.nlf_lu_inverse_elems(n), dtype=torch.complex128, device="cuda")
    nl.nlf_lu_block_inverses(A, dinv)
    X2 = torch.empty((batch, 8, n), dtype=torch.complex128, device="cuda")
    tmp = torch.empty(batch * 256 * 8, dtype=torch.complex128, device="cuda")
    nl.nlf_getrs_batched_inv(A, perm, dinv, dev(B), X2, tmp, shared_rhs=True)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0, 0]
    for b in range(batch):
        for XX in (X, X2):
            x = nl.from_colmajor(XX[b])
            r = mats[b] @ x - B
            berr = np.linalg.norm(r) / (np.linalg.norm(mats[b]) * np.linalg.norm(x) + np.linalg.norm(B))
            assert berr < 1e-14, berr
        assert np.array_equal(np.sort(perm[b].cpu().numpy()), np.arange(n))


@pytest.mark.parametrize("n,m,nz", [(333, 11, 6), (333, 11, 19), (700, 200, 7), (1030, 520, 5)])
def test_accumulate_matches_oracle(n, m, nz):
    # the three launch forms by block size: one row per thread and eight nodes per load batch,
    # two rows and four nodes (700 x 200), four rows and one node (1030 x 520: 1040
    # workgroups); ragged row slabs and node tails in each
    rng = np.random.default_rng(5 + nz)
    X = wl.cn(rng, (n, m))
    Ys = [wl.cn(rng, (n, m)) for _ in range(nz)]
    C = qd.Contour(0.1, 0.5)
    z, w = qd.nodes_weights(C, nz)
    lam = 0.2 * wl.cn(rng, m)
    Q = torch.empty((m, n), dtype=torch.complex128, device="cuda")
    nl.nlf_accumulate(dev(X), batch_dev(Ys), z, w, lam, Q)
    torch.cuda.synchronize()
    assert rel(nl.from_colmajor(Q), dense.step4_sum(X, Ys, lam, z, w)) < 1e-13


def test_block_residual_matches_oracle():
    rng = np.random.default_rng(6)
    n, m = 257, 9
    terms = wl.DELAY
    mats = [wl.cn(rng, (n, n)) for _ in terms]
    X = wl.cn(rng, (n, m))
    lam = 0.3 * wl.cn(rng, m)
    R = torch.empty((m, n), dtype=torch.complex128, device="cuda")
    norms = torch.empty(m, dtype=torch.float64, device="cuda")
    ws = torch.empty((m, n), dtype=torch.complex128, device="cuda")
    nl.nlf_block_residual(terms, [dev(M) for M in mats], dev(X), lam, R, norms, ws)
    torch.cuda.synchronize()
    R0, n0 = dense.block_residual(terms, mats, X, lam)
    assert rel(nl.from_colmajor(R), R0) < 1e-13
    assert rel(norms.cpu().numpy(), n0) < 1e-13


def test_project_matches_oracle():
    rng = np.random.default_rng(7)
    n, m = 700, 24
    mats = [wl.cn(rng, (n, n)) for _ in range(3)]
    Q, _ = np.linalg.qr(wl.cn(rng, (n, m)))
    W = torch.empty((3 * m, n), dtype=torch.complex128, device="cuda")
    Ah = torch.empty((3, m, m), dtype=torch.complex128, device="cuda")
    ws = torch.empty(nl.nlf_project_workspace(n, m, 3), dtype=torch.complex128, device="cuda")
    nl.nlf_project([dev(M) for M in mats], dev(Q), W, Ah, ws)
    torch.cuda.synchronize()
    ref = dense.project(mats, Q)
    for j in range(3):
        assert rel(nl.from_colmajor(Ah[j]), ref[j]) < 1e-13


def test_project_long_reduction_matches_definition():
    # n = 4096, m = 160: W_j = A_j Q has a 4096-long reduction into 192 output tiles of 64 x 64,
    # which the library runs as split-K partial products (direct-to-LDS 3M tile) summed by a
    # reduction kernel; W_j itself and Ahat_j = Q^H W_j against their definitions
    rng = np.random.default_rng(11)
    n, m, J = 4096, 160, 2
    mats = [wl.cn(rng, (n, n)) / np.sqrt(n) for _ in range(J)]
    Q, _ = np.linalg.qr(wl.cn(rng, (n, m)))
    W = torch.empty((J * m, n), dtype=torch.complex128, device="cuda")
    Ah = torch.empty((J, m, m), dtype=torch.complex128, device="cuda")
    ws = torch.empty(nl.nlf_project_workspace(n, m, J), dtype=torch.complex128, device="cuda")
    nl.nlf_project([dev(M) for M in mats], dev(Q), W, Ah, ws)
    torch.cuda.synchronize()
    Wh = nl.from_colmajor(W)
    for j in range(J):
        Wj = mats[j] @ Q
        assert rel(Wh[:, j * m:(j + 1) * m], Wj) < 1e-13 * np.sqrt(n)
        assert rel(nl.from_colmajor(Ah[j]), Q.conj().T @ Wj) < 1e-13 * np.sqrt(n)


@pytest.mark.parametrize("n,m", [(1500, 45), (300, 64)])
def test_orthonormalize_rank_deficient_block(n, m):
    # singular values from 1 down to 1e-20: the Gram matrix is numerically singular, so the
    # block goes through the Householder path (ragged last panel at m = 45); the result must
    # be orthonormal and contain every direction whose singular value is at least 1e-6
    rng = np.random.default_rng(9)
    U, _ = np.linalg.qr(wl.cn(rng, (n, m)))
    Vh, _ = np.linalg.qr(wl.cn(rng, (m, m)))
    s = np.logspace(0, -20, m)
    Q0 = (U * s[None, :]) @ Vh
    Q = dev(Q0)
    ws = torch.empty(nl.nlf_orth_workspace(n, m), dtype=torch.complex128, device="cuda")
    nl.nlf_orthonormalize(Q, ws)
    torch.cuda.synchronize()
    q = nl.from_colmajor(Q)
    assert np.all(np.isfinite(q))
    assert np.max(np.abs(q.conj().T @ q - np.eye(m))) < 1e-13
    k = int(np.sum(s >= 1e-6))
    Uk = U[:, :k]
    assert np.max(np.abs(q @ (q.conj().T @ Uk) - Uk)) < 1e-8
    # the leading columns span what the leading columns of Q0 span (a QR factorisation)
    ref, _ = np.linalg.qr(Q0[:, :4])
    assert np.max(np.abs(q[:, :4] @ (q[:, :4].conj().T @ ref) - ref)) < 1e-12


def test_orthonormalize_keeps_span():
    rng = np.random.default_rng(8)
    n, m = 2000, 40
    Q0 = wl.cn(rng, (n, m)) @ np.diag(np.logspace(0, -6, m))     # ill-conditioned columns
    Q = dev(Q0)
    ws = torch.empty(nl.nlf_orth_workspace(n, m), dtype=torch.complex128, device="cuda")
    nl.nlf_orthonormalize(Q, ws)
    torch.cuda.synchronize()
    q = nl.from_colmajor(Q)
    assert np.max(np.abs(q.conj().T @ q - np.eye(m))) < 1e-13
    ref, _ = np.linalg.qr(Q0)
    # same column space: the projector onto span(Q0) reproduces q
    assert np.max(np.abs(ref @ (ref.conj().T @ q) - q)) < 1e-11


@pytest.mark.parametrize("dtype", ["c128", "c64"])
@pytest.mark.parametrize("M,N,K,batch", [(2048, 96, 256, 24), (1000, 70, 64, 8)])
def test_gemm_forced_32_column_tile_matches_definition(dtype, M, N, K, batch):
    # products on the 32-column tiles through the explicit-tile entry point (64 x 32 for
    # complex128, 128 x 32 for complex64): the direct-to-LDS forms, full and ragged, against the
    # plain definition
    rng = np.random.default_rng(M + N + K)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    tol = 1e-13 if dtype == "c128" else 2e-5
    A = [wl.cn(rng, (M, K)) for _ in range(batch)]
    B = [wl.cn(rng, (K, N)) for _ in range(batch)]
    C = [wl.cn(rng, (M, N)) for _ in range(batch)]
    if dtype == "c64":
        A, B, C = ([X.astype(np.complex64).astype(complex) for X in Y] for Y in (A, B, C))
    alpha, beta = 0.5 + 0.5j, -1.0
    Ad, Bd, Cd = batch_dev(A, dt), batch_dev(B, dt), batch_dev(C, dt)
    tm, tn = (2, 1) if dtype == "c128" else (4, 1)
    nl.nlf_gemm_batched_tile("N", M, N, K, alpha, Ad, M, M * K, Bd, K, K * N, beta, Cd, M, M * N, batch, tm, tn)
    torch.cuda.synchronize()
    for b in range(batch):
        ref = alpha * (A[b] @ B[b]) + beta * C[b]
        assert rel(nl.from_colmajor(Cd[b]).astype(complex), ref) < tol * np.sqrt(K)


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_getrf_ragged_tiles_backward_error(dtype):
    # n = 2000 = 31 x 64 + 16, 4 matrices: the trailing updates and U12 products have ragged
    # 64 x 64 (complex128) and 128 x 64 (complex64) tiles, the predicated direct-to-LDS forms,
    # from the first panel on; P A = L U to working accuracy and a valid permutation
    n, batch = 2000, 4
    rng = np.random.default_rng(2000)
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    eps = 2.2e-16 if dtype == "c128" else 1.2e-7
    mats = [wl.cn(rng, (n, n)) / np.sqrt(n) for _ in range(batch)]
    if dtype == "c64":
        mats = [M.astype(np.complex64).astype(complex) for M in mats]
    A = batch_dev(mats, dt)
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    dinv = torch.empty(batch * nl.nlf_lu_inverse_elems(n), dtype=dt, device="cuda")
    nl.nlf_getrf_batched_blocked(A, ipiv, perm, info, dinv)
    torch.cuda.synchronize()
    assert info.cpu().numpy().tolist() == [0] * batch
    for b in range(batch):
        LU = nl.from_colmajor(A[b]).astype(complex)
        L = np.tril(LU, -1) + np.eye(n)
        U = np.triu(LU)
        p = perm[b].cpu().numpy()
        assert np.array_equal(np.sort(p), np.arange(n))
        err = np.max(np.abs(mats[b][p] - L @ U)) / np.max(np.abs(mats[b]))
        assert err < 30 * n * eps, err


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_getrf_headline_shape_sampled_rows(dtype):
    # the benchmarked factorisation shape and launch sequence: 24 matrices of n = 8192 (the
    # headline's node count and order), factored by the blocked LU.  A property that holds at any
    # size, checked on sampled rows: row i of L U equals row perm[i] of A to working accuracy;
    # perm is a permutation and |l_ij| <= sqrt(2) (partial pivoting on |Re| + |Im|, which bounds
    # the modulus of a multiplier by sqrt(2)).  A is regenerated from its seed
    # rather than kept, so only the factors occupy the device.
    n, batch = 8192, 24
    dt = torch.complex128 if dtype == "c128" else torch.complex64
    eps = 2.2e-16 if dtype == "c128" else 1.2e-7

    def gen():
        g = torch.Generator(device="cuda").manual_seed(8192)
        return torch.randn((batch, n, n), dtype=dt, device="cuda", generator=g)

    F = gen()            # (batch, n, n) storage read as column-major: matrix b is F[b].T
    ipiv = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    perm = torch.empty((batch, n), dtype=torch.int32, device="cuda")
    info = torch.empty(batch, dtype=torch.int32, device="cuda")
    dinv = torch.empty(batch * nl.nlf_lu_inverse_elems(n), dtype=dt, device="cuda")
    nl.nlf_getrf_batched_blocked(F, ipiv, perm, info, dinv)
    torch.cuda.synchronize()
    del dinv
    assert info.cpu().numpy().tolist() == [0] * batch
    rng = np.random.default_rng(24)
    rows = np.unique(np.concatenate([[0, 1, 511, 512, 4095, 7679, 7680, n - 1],
                                     rng.choice(n, 8, replace=False)]))
    ri = torch.as_tensor(rows, device="cuda")
    G = gen()
    for b in range(batch):
        p = perm[b].cpu().numpy()
        assert np.array_equal(np.sort(p), np.arange(n))
        LU = F[b].T                                  # the factors, row-major view
        Lfull = torch.tril(LU, -1)
        assert float(Lfull.abs().max()) <= np.sqrt(2.0) * (1 + 4 * eps)
        del Lfull
        # the sampled rows of L: entries left of the diagonal, and the unit diagonal
        cols = torch.arange(n, device="cuda")
        Lr = torch.where(cols[None, :] < ri[:, None], LU[ri], torch.zeros((), dtype=dt, device="cuda"))
        Lr[torch.arange(len(rows), device="cuda"), ri] = 1
        U = torch.triu(LU)
        got = (Lr.to(torch.complex128) @ U.to(torch.complex128)).cpu().numpy()
        del U
        Ab = G[b].T                                  # matrix b
        want = Ab[torch.as_tensor(p[rows].astype(np.int64), device="cuda")].to(torch.complex128).cpu().numpy()
        scale = float(Ab.abs().max())
        err = np.max(np.abs(got - want)) / scale
        assert err < 30 * n * eps, (b, err)
    del F, G
    torch.cuda.empty_cache()      # 2 x 26 GB (complex128) back to the device for the later tests
