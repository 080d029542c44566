"""Kernel-level GPU parity: the gathered MFMA GEMM, CholeskyQR
orthogonalization, the one-sided Jacobi small SVD and one zip-up operator
application, each against plain CPU arithmetic (numpy / the oracle)."""
import ctypes as C

import numpy as np
import pytest

from oracle import rsvd
from oracle.network import zipup_operator

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def _rand(rng, shape, cplx):
    x = rng.standard_normal(shape)
    if cplx:
        x = x + 1j * rng.standard_normal(shape)
    return x


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _p(t):
    return C.c_void_p(t.data_ptr())


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("shape", [(1, 1, 1), (16, 16, 4), (17, 33, 5), (64, 64, 64), (130, 47, 300),
                                   (44, 44, 1296), (3, 200, 7), (1296, 44, 44)])
@pytest.mark.parametrize("trans", [0, 1])
def test_gemm(ctx, cplx, shape, trans):
    M, N, K = shape
    rng = np.random.default_rng(M * 1000 + N * 10 + K)
    B = 2
    A = _rand(rng, (B, K, M) if trans else (B, M, K), cplx)
    Bm = _rand(rng, (B, K, N), cplx)
    dA, dB = _dev(A), _dev(Bm)
    dC = torch.zeros((B, M, N), dtype=dA.dtype, device="cuda")
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_gemm(ctx.h, hp.C128 if cplx else hp.F64, B, M, N, K, trans,
                                      _p(dA), _p(dB), _p(dC)))
    out = dC.cpu().numpy()
    for b in range(B):
        opA = A[b].conj().T if trans else A[b]
        ref = opA @ Bm[b]
        assert np.max(np.abs(out[b] - ref)) <= 1e-13 * max(1.0, np.abs(ref).max()) * np.sqrt(K)


N_TILES = 15  # tile shapes of the GEMM (0..14; complex products use those of <= 4 tiles per wave)


@pytest.mark.parametrize("tile", range(N_TILES))
@pytest.mark.parametrize("kstep,split", [(1, 1), (2, 1), (1, 3), (2, 0)])
def test_gemm_every_variant(ctx, tile, kstep, split):
    """Each kernel instantiation (tile shape x K-step x split-K), forced through the
    variant hook on a ragged batched product (several tiles, partial edge tiles,
    a K tail), real and complex, both operand layouts."""
    rng = np.random.default_rng(tile * 10 + kstep + split)
    B, M, N, K = 2, 230, 150, 77
    try:
        ctx.check(ctx.lib.hpeps_test_gemm_variant(ctx.h, tile, kstep, split))
        for cplx in (False, True):
            for trans in (0, 1):
                A = _rand(rng, (B, K, M) if trans else (B, M, K), cplx)
                Bm = _rand(rng, (B, K, N), cplx)
                dA, dB = _dev(A), _dev(Bm)
                dC = torch.zeros((B, M, N), dtype=dA.dtype, device="cuda")
                ctx.sync_stream()
                ctx.check(ctx.lib.hpeps_test_gemm(ctx.h, hp.C128 if cplx else hp.F64, B, M, N, K, trans,
                                                  _p(dA), _p(dB), _p(dC)))
                out = dC.cpu().numpy()
                for b in range(B):
                    ref = (A[b].conj().T if trans else A[b]) @ Bm[b]
                    assert np.max(np.abs(out[b] - ref)) <= 1e-13 * np.abs(ref).max() * np.sqrt(K)
    finally:
        ctx.check(ctx.lib.hpeps_test_gemm_variant(ctx.h, -1, 1, 0))


@pytest.mark.parametrize("smallk", [1, 0])
@pytest.mark.parametrize("shape", [(17, 300, 5), (8, 1030, 16), (40, 513, 1), (72, 9504, 6), (9, 777, 12),
                                   (6, 9504, 72), (3, 1030, 200), (8, 512, 17), (1, 2050, 9),
                                   (300, 36, 12), (130, 96, 16), (40, 72, 6), (5, 20, 3), (260, 80, 2)])
@pytest.mark.parametrize("trans", [0, 1])
def test_gemm_skinny(ctx, smallk, shape, trans):
    """Real skinny products: K <= 16 (the store-bound kernel, wide rows and rows narrower than
    one pass of column groups) and M <= 8 with N >= 256 (the read-bound kernel), and with them
    switched off the MFMA tile kernel: ragged rows and column chunks, K = 1, K past 8, K not a
    multiple of the 8-deep load batch, M = 1, more rows than one work item holds."""
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N + K)
    B = 3
    A = rng.standard_normal((B, K, M) if trans else (B, M, K))
    Bm = rng.standard_normal((B, K, N))
    dA, dB = _dev(A), _dev(Bm)
    dC = torch.full((B, M, N), np.nan, dtype=torch.float64, device="cuda")
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_gemm_smallk(ctx.h, smallk))
    try:
        ctx.check(ctx.lib.hpeps_test_gemm(ctx.h, hp.F64, B, M, N, K, trans, _p(dA), _p(dB), _p(dC)))
    finally:
        ctx.check(ctx.lib.hpeps_test_gemm_smallk(ctx.h, 1))
    out = dC.cpu().numpy()
    for b in range(B):
        ref = (A[b].T if trans else A[b]) @ Bm[b]
        assert np.max(np.abs(out[b] - ref)) <= 1e-14 * max(1.0, np.abs(ref).max()) * K


def test_profile_by_shape(ctx):
    """Live timing keeps GEMM classes apart by product shape when asked to, and counts the
    algorithmic work of each product (2 M N K flops per instance)."""
    rng = np.random.default_rng(5)
    B = 3
    shapes = [(40, 70, 9), (33, 20, 50)]
    bufs = []
    for M, N, K in shapes:
        bufs.append((_dev(rng.standard_normal((B, M, K))), _dev(rng.standard_normal((B, K, N))),
                     torch.zeros((B, M, N), dtype=torch.float64, device="cuda")))
    ctx.sync_stream()
    for by_shape in (True, False):
        hp.profile_by_shape(ctx, by_shape)
        hp.profile_start(ctx, "gemm_f64")
        for (M, N, K), (dA, dB, dC) in zip(shapes, bufs):
            ctx.check(ctx.lib.hpeps_test_gemm(ctx.h, hp.F64, B, M, N, K, 0, _p(dA), _p(dB), _p(dC)))
        agg = hp.profile_read(ctx)
        hp.profile_stop(ctx)
        if by_shape:
            for M, N, K in shapes:
                names = [n for n in agg if n.endswith(f"_M{M}_N{N}_K{K}_b{B}")]
                assert len(names) == 1, agg.keys()
                a = agg[names[0]]
                assert a["launches"] == 1 and a["ms"] > 0
                assert a["flops"] == pytest.approx(2.0 * M * N * K * B)
        else:
            assert all("_M" not in n for n in agg)
            assert sum(a["launches"] for a in agg.values()) == len(shapes)
    hp.profile_by_shape(ctx, False)


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("nk", [(8, 8), (100, 7), (1296, 44), (5000, 108), (300, 128)])
def test_orthogonalize(ctx, cplx, nk):
    n, k = nk
    if cplx and k > 88:
        pytest.skip("complex small factorizations are limited to k <= 88")
    rng = np.random.default_rng(n + k)
    B = 2
    Y = _rand(rng, (B, n, k), cplx)
    dY = _dev(Y)
    dP = torch.zeros_like(dY)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_orthogonalize(ctx.h, hp.C128 if cplx else hp.F64, B, n, k,
                                               _p(dY), _p(dP)))
    P = dP.cpu().numpy()
    for b in range(B):
        assert np.max(np.abs(P[b].conj().T @ P[b] - np.eye(k))) < 1e-13
        # same range: the projector onto range(Y) fixes Y
        Q = np.linalg.qr(Y[b])[0]
        assert np.max(np.abs(P[b] @ (P[b].conj().T @ Q) - Q)) < 1e-12


def _orth_eigh(ctx, Y, cplx):
    B, n, k = Y.shape
    dY = _dev(Y)
    dP = torch.zeros_like(dY)
    dR = torch.zeros((B, k, k), dtype=dY.dtype, device=dY.device)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_orthogonalize_eigh(ctx.h, hp.C128 if cplx else hp.F64, B, n, k,
                                                    _p(dY), _p(dP), _p(dR)))
    assert np.array_equal(dY.cpu().numpy(), Y)  # input left intact
    return dP.cpu().numpy(), dR.cpu().numpy()


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("nk", [(8, 8), (100, 7), (1296, 44), (5000, 108), (300, 128)])
def test_orthogonalize_eigh(ctx, cplx, nk):
    """Alg. 5 (two passes, first shifted) against the oracle's single pass on
    well-conditioned panels: same range (equal projectors), Q^H Q = I,
    Q R = Y and R^H R = Y^H Y."""
    n, k = nk
    if cplx and k > 88:
        pytest.skip("complex small factorizations are limited to k <= 88")
    rng = np.random.default_rng(3 * n + k)
    B = 2
    Y = _rand(rng, (B, n, k), cplx)
    P, R = _orth_eigh(ctx, Y, cplx)
    for b in range(B):
        Qo, Ro = rsvd.orthogonalize_gram_eigh(Y[b])
        nrm = np.max(np.abs(Y[b]))
        assert np.max(np.abs(P[b].conj().T @ P[b] - np.eye(k))) < 1e-13
        assert np.max(np.abs(P[b] @ P[b].conj().T - Qo @ Qo.conj().T)) < 1e-12
        assert np.max(np.abs(P[b] @ R[b] - Y[b])) < 1e-13 * k * nrm
        G = Ro.conj().T @ Ro
        assert np.max(np.abs(R[b].conj().T @ R[b] - G)) < 1e-12 * np.max(np.abs(G))


def test_orthogonalize_eigh_ill_conditioned(ctx):
    """kappa(Y) = 1e6 (kappa(G) = 1e12): one unshifted pass of Alg. 5 leaves Q
    far from orthonormal (the oracle's single pass shows it); the shifted
    second pass restores orthonormality and Q R = Y."""
    rng = np.random.default_rng(4)
    n, k = 2000, 40
    U = np.linalg.qr(rng.standard_normal((n, k)))[0]
    V = np.linalg.qr(rng.standard_normal((k, k)))[0]
    Y = (U * np.logspace(0, -6, k)) @ V.T
    Qo, _ = rsvd.orthogonalize_gram_eigh(Y)
    assert np.max(np.abs(Qo.T @ Qo - np.eye(k))) > 1e-8
    P, R = _orth_eigh(ctx, Y[None], False)
    assert np.max(np.abs(P[0].T @ P[0] - np.eye(k))) < 1e-12
    assert np.max(np.abs(P[0] @ R[0] - Y)) < 1e-13
    assert np.max(np.abs(P[0] @ (P[0].T @ U) - U)) < 1e-9


@pytest.mark.parametrize("cplx", [False, True])
def test_orthogonalize_eigh_rank_deficient(ctx, cplx):
    """Exact rank 9 in a 13-column panel: the Gram-based passes cannot
    resolve the null directions, the Householder fallback replaces the panel;
    Q is still orthonormal with Q R = Y."""
    rng = np.random.default_rng(6)
    n, k, r = 500, 13, 9
    Y = (_rand(rng, (n, r), cplx) @ _rand(rng, (r, k), cplx))[None]
    P, R = _orth_eigh(ctx, Y, cplx)
    assert hp.get_info(ctx)["orth_householder"] >= 1
    assert np.max(np.abs(P[0].conj().T @ P[0] - np.eye(k))) < 1e-13
    assert np.max(np.abs(P[0] @ R[0] - Y[0])) < 1e-13 * np.max(np.abs(Y))


def test_orthogonalize_ill_conditioned(ctx):
    """kappa ~ 1e12: the shifted first pass plus a third pass still orthonormalize."""
    rng = np.random.default_rng(0)
    n, k = 2000, 40
    U = np.linalg.qr(rng.standard_normal((n, k)))[0]
    V = np.linalg.qr(rng.standard_normal((k, k)))[0]
    Y = (U * np.logspace(0, -12, k)) @ V.T
    dY = _dev(Y[None])
    dP = torch.zeros_like(dY)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_orthogonalize(ctx.h, hp.F64, 1, n, k, _p(dY), _p(dP)))
    P = dP.cpu().numpy()[0]
    info = hp.get_info(ctx)
    assert info["orth_extra_passes"] >= 1
    assert np.max(np.abs(P.T @ P - np.eye(k))) < 1e-12
    # leading directions (well above the shift) are reproduced
    lead = U[:, :20]
    assert np.max(np.abs(P @ (P.T @ lead) - lead)) < 1e-8


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("k", [1, 2, 7, 44, 108])
def test_small_svd(ctx, cplx, k):
    if cplx and k > 88:
        pytest.skip("complex small factorizations are limited to k <= 88")
    rng = np.random.default_rng(k)
    B = 2
    R = np.triu(_rand(rng, (B, k, k), cplx))
    dR = _dev(R)
    dZ = torch.zeros_like(dR)
    ds = torch.zeros((B, k), dtype=torch.float64, device="cuda")
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_small_svd(ctx.h, hp.C128 if cplx else hp.F64, B, k, _p(dR), _p(dZ),
                                           _p(ds)))
    Z, s = dZ.cpu().numpy(), ds.cpu().numpy()
    for b in range(B):
        K = R[b].conj().T
        ref = np.linalg.svd(K, compute_uv=False)
        assert np.max(np.abs(s[b] - ref)) < 1e-13 * ref[0] * k
        assert np.max(np.abs(Z[b].conj().T @ Z[b] - np.eye(k))) < 1e-12
        # Z spans the left singular subspaces: Z^H K K^H Z = diag(s^2)
        M = Z[b].conj().T @ K @ K.conj().T @ Z[b]
        assert np.max(np.abs(M - np.diag(s[b] ** 2))) < 1e-12 * ref[0] ** 2 * k


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("k", [16, 44, 108])
def test_small_svd_near_identity(ctx, cplx, k):
    """R = I + rounding-level noise (the factor of an already orthonormal
    panel): every rotation is decided at the noise level, so the lanes that
    share a column pair must agree bit for bit on the pair's inner products.
    The singular values stay within a few eps of 1."""
    if cplx and k > 88:
        pytest.skip("complex small factorizations are limited to k <= 88")
    rng = np.random.default_rng(100 + k)
    B = 4
    R = np.triu(_rand(rng, (B, k, k), cplx)) * 1e-15 + np.eye(k)
    dR = _dev(R)
    dZ = torch.zeros_like(dR)
    ds = torch.zeros((B, k), dtype=torch.float64, device="cuda")
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_small_svd(ctx.h, hp.C128 if cplx else hp.F64, B, k, _p(dR), _p(dZ),
                                           _p(ds)))
    Z, s = dZ.cpu().numpy(), ds.cpu().numpy()
    for b in range(B):
        K = R[b].conj().T
        assert np.max(np.abs(s[b] - np.linalg.svd(K, compute_uv=False))) < 1e-13
        M = Z[b].conj().T @ K @ K.conj().T @ Z[b]
        assert np.max(np.abs(M - np.diag(s[b] ** 2))) < 1e-13


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("dims", [(1, 2, 1, 2, 2, 3, 2, 2, 2), (3, 2, 2, 3, 2, 4, 2, 1, 2),
                                  (5, 3, 4, 2, 3, 5, 3, 2, 2)])
@pytest.mark.parametrize("order", [0, 1, 2])
def test_zip_apply(ctx, cplx, dims, order):
    """A X and A^* P of the zip-up operator in each contraction order of the middle
    stages (0: cost-model choice, 1: bra then boundary, 2: boundary then bra)."""
    ctx.check(ctx.lib.hpeps_test_zip_order(ctx.h, order))
    try:
        _zip_apply_case(ctx, cplx, dims)
    finally:
        ctx.check(ctx.lib.hpeps_test_zip_order(ctx.h, 0))


def _zip_apply_case(ctx, cplx, dims):
    a, x, b, h, u, c, y, g, d = dims
    rng = np.random.default_rng(sum(dims))
    V = _rand(rng, (a, x, x, b, h, h), cplx)
    S = _rand(rng, (b, u, u, c), cplx)
    T = _rand(rng, (u, y, h, g, d), cplx)
    Bra = _rand(rng, (u, y, h, g, d), cplx)
    op = zipup_operator(V, S, T, Bra)
    k = 5
    X = _rand(rng, (op.n_cols, k), cplx)
    P = _rand(rng, (op.n_rows, k), cplx)
    dd = (C.c_int64 * 9)(*dims)
    dt = hp.C128 if cplx else hp.F64
    tV, tS, tT, tB = _dev(V[None]), _dev(S[None]), _dev(T[None]), _dev(Bra[None])
    dX, dP = _dev(X[None]), _dev(P[None])
    dY = torch.zeros((1, op.n_rows, k), dtype=dX.dtype, device="cuda")
    dZ = torch.zeros((1, op.n_cols, k), dtype=dX.dtype, device="cuda")
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_zip_apply(ctx.h, dt, 1, dd, _p(tV), _p(tS), _p(tT), _p(tB), k, 0,
                                           _p(dX), _p(dY)))
    ctx.check(ctx.lib.hpeps_test_zip_apply(ctx.h, dt, 1, dd, _p(tV), _p(tS), _p(tT), _p(tB), k, 1,
                                           _p(dP), _p(dZ)))
    Y, Z = dY.cpu().numpy()[0], dZ.cpu().numpy()[0]
    ry, rz = op.apply(X), op.apply_adj(P)
    assert np.max(np.abs(Y - ry)) < 1e-12 * np.abs(ry).max()
    assert np.max(np.abs(Z - rz)) < 1e-12 * np.abs(rz).max()


def _householder(ctx, Y, cplx):
    B, n, k = Y.shape
    dY = _dev(Y)
    dP = torch.zeros_like(dY)
    dR = torch.full((B, k, k), 7.0, dtype=dY.dtype, device="cuda")
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_householder(ctx.h, hp.C128 if cplx else hp.F64, B, n, k,
                                             _p(dY), _p(dP), _p(dR)))
    assert np.array_equal(dY.cpu().numpy(), Y)
    return dP.cpu().numpy(), dR.cpu().numpy()


@pytest.mark.parametrize("n,k,cplx,B", [(50, 7, False, 2), (300, 9, True, 1), (37, 37, True, 1),
                                        (4000, 44, False, 3), (20000, 108, False, 1), (3000, 88, True, 1),
                                        (129, 64, False, 2)])
def test_householder_qr(ctx, n, k, cplx, B):
    """Householder TSQR (the orthogonalization fallback).  Full-rank panels: Q orthonormal,
    Q R = Y, R upper triangular and equal to LAPACK's R up to the signs of its rows (Q to
    LAPACK's Q up to the same column signs).  Rank-deficient panels (an exactly zero and a
    duplicated column): Q orthonormal, Q R = Y; with one row block (n < 4k) and only the zero
    column, Q and R equal LAPACK's, reflector convention included (tau = 0 on the zero
    column)."""
    rng = np.random.default_rng(n + k)
    Y = rng.standard_normal((B, n, k))
    if cplx:
        Y = Y + 1j * rng.standard_normal((B, n, k))
    P, R = _householder(ctx, Y, cplx)
    for b in range(B):
        nrm = np.linalg.norm(Y[b], 2)
        assert np.max(np.abs(P[b].conj().T @ P[b] - np.eye(k))) < 1e-13
        assert np.max(np.abs(P[b] @ R[b] - Y[b])) < 1e-13 * nrm
        assert np.all(np.tril(R[b], -1) == 0)
        Q0, R0 = np.linalg.qr(Y[b])
        ph = np.diag(R[b]) / np.diag(R0)             # unit-modulus row factors
        assert np.max(np.abs(np.abs(ph) - 1)) < 1e-12
        assert np.max(np.abs(R[b] - ph[:, None] * R0)) < 1e-12 * nrm
        assert np.max(np.abs(P[b] - Q0 * ph.conj()[None, :])) < 1e-11
    Yz = Y.copy()
    Yz[:, :, 3] = 0
    P, R = _householder(ctx, Yz, cplx)
    for b in range(B):
        assert np.max(np.abs(P[b].conj().T @ P[b] - np.eye(k))) < 1e-13
        assert np.max(np.abs(P[b] @ R[b] - Yz[b])) < 1e-13 * np.linalg.norm(Yz[b], 2)
        if n < 4 * k:
            Q0, R0 = np.linalg.qr(Yz[b])
            assert np.max(np.abs(P[b] - Q0)) < 1e-12
            assert np.max(np.abs(R[b] - R0)) < 1e-12 * np.linalg.norm(Yz[b], 2)
    Yd = Yz.copy()
    Yd[:, :, 5] = Yd[:, :, 1]
    P, R = _householder(ctx, Yd, cplx)
    for b in range(B):
        assert np.max(np.abs(P[b].conj().T @ P[b] - np.eye(k))) < 1e-13
        assert np.max(np.abs(P[b] @ R[b] - Yd[b])) < 1e-13 * np.linalg.norm(Yd[b], 2)
        assert np.all(np.tril(R[b], -1) == 0)


def test_orthogonalize_rank_deficient_uses_householder(ctx):
    """A panel of exact rank 10 < k = 24: the first Cholesky pass flags it, the Householder
    fallback produces P, and P is orthonormal with range(P) containing range(Y) to rounding."""
    rng = np.random.default_rng(3)
    n, k, r = 3000, 24, 10
    Y = rng.standard_normal((n, r)) @ rng.standard_normal((r, k))
    dY = _dev(Y[None])
    dP = torch.zeros_like(dY)
    hp.get_info(ctx)
    ctx.sync_stream()
    ctx.check(ctx.lib.hpeps_test_orthogonalize(ctx.h, hp.F64, 1, n, k, _p(dY), _p(dP)))
    info = hp.get_info(ctx)
    assert info["orth_householder"] == 1
    P = dP.cpu().numpy()[0]
    assert np.max(np.abs(P.T @ P - np.eye(k))) < 1e-13
    assert np.linalg.norm(Y - P @ (P.T @ Y)) < 1e-14 * np.linalg.norm(Y)
