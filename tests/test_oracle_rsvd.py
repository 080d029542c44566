"""Pins of the oracle's sketch generator and einsumsvd (definition and Alg. 4)."""
import os

import numpy as np
import pytest

import synth
from oracle import rsvd
from oracle.network import pair_operator, zipup_operator
from oracle.sketch import mix64, sketch

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_splitmix64_reference_vector():
    vals = [int(l) for l in open(os.path.join(GOLDEN, "splitmix64_seed1234567.txt"))
            if l.strip() and not l.startswith("#")]
    phi = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        got = [int(mix64(np.uint64(1234567) + np.uint64(i + 1) * phi)) for i in range(5)]
    assert got == vals


def test_sketch_range_and_moments():
    om = sketch(7, 3, 5000, 40)
    assert om.dtype == np.float64 and om.shape == (5000, 40)
    assert om.min() >= -1.0 and om.max() < 1.0
    # uniform on [-1, 1): mean 0, variance 1/3 (loose statistical bounds)
    assert abs(om.mean()) < 0.01 and abs(om.var() - 1 / 3) < 0.01
    # values lie on the 2^-52 grid, so x = (om + 1) * 2^52 is an integer < 2^53
    x = (om + 1.0) * 2.0 ** 52
    assert np.all(x == np.floor(x)) and x.max() < 2.0 ** 53


def test_sketch_streams_differ_and_repeat():
    a = sketch(1, 5, 10, 4)
    assert np.array_equal(a, sketch(1, 5, 10, 4))
    assert not np.array_equal(a, sketch(1, 6, 10, 4))
    assert not np.array_equal(a, sketch(2, 5, 10, 4))
    # prefix property: element i does not depend on the total size
    b = sketch(1, 5, 20, 4)
    assert np.array_equal(a, b[:10])


def _rand(shape, rng, complex_):
    x = rng.standard_normal(shape)
    if complex_:
        x = x + 1j * rng.standard_normal(shape)
    return x


def test_truncated_svd_eckart_young():
    rng = np.random.default_rng(0)
    A = rng.standard_normal((30, 20)) @ np.diag(0.7 ** np.arange(20)) @ rng.standard_normal((20, 25))
    full = np.linalg.svd(A, compute_uv=False)
    for m in (1, 5, 12):
        U, s, Vh = rsvd.truncated_svd(A, m)
        R = A - (U * s) @ Vh
        assert np.isclose(np.linalg.norm(R) ** 2, np.sum(full[m:] ** 2), rtol=1e-10)
        assert np.isclose(np.linalg.norm(R, 2), full[m], rtol=1e-10)
        assert np.allclose(U.T @ U, np.eye(m), atol=1e-13)
        assert np.allclose(Vh @ Vh.T, np.eye(m), atol=1e-13)
        assert np.all(np.diff(s) <= 0)


def _zip_inputs(rng, a, x, b, h, u, c, y, g, d, complex_):
    V = _rand((a, x, x, b, h, h), rng, complex_)
    S = _rand((b, u, u, c), rng, complex_)
    T = _rand((u, y, h, g, d), rng, complex_)
    B = _rand((u, y, h, g, d), rng, complex_)
    return V, S, T, B


@pytest.mark.parametrize("complex_", [False, True])
def test_operator_adjoint_identity(complex_):
    """<Y, A X> = <A^* Y, X>, and the implicit products equal the explicit matrix."""
    rng = np.random.default_rng(1)
    op = zipup_operator(*_zip_inputs(rng, 3, 2, 2, 2, 2, 3, 2, 2, 2, complex_))
    X = _rand((op.n_cols, 5), rng, complex_)
    Y = _rand((op.n_rows, 5), rng, complex_)
    lhs = np.vdot(Y, op.apply(X))
    rhs = np.vdot(op.apply_adj(Y), X)
    assert np.isclose(lhs, rhs, rtol=1e-12)
    A = op.explicit()
    assert np.allclose(op.apply(X), A @ X, rtol=1e-12, atol=1e-12)
    assert np.allclose(op.apply_adj(Y), A.conj().T @ Y, rtol=1e-12, atol=1e-12)


def test_zipup_operator_by_loops():
    """Brute-force sum over every index on a tiny case."""
    rng = np.random.default_rng(2)
    V, S, T, B = _zip_inputs(rng, 2, 2, 1, 2, 2, 2, 1, 2, 2, True)
    op = zipup_operator(V, S, T, B)
    A = op.explicit().reshape(op.rows_shape + op.cols_shape)
    ref = np.zeros_like(A)
    it = np.ndindex
    for (a, x, X) in it(*op.rows_shape):
        for (y, Y, c, g, G) in it(*op.cols_shape):
            acc = 0
            for (b, h, H, u, U, p) in it(V.shape[3], V.shape[4], V.shape[5], S.shape[1],
                                         S.shape[2], T.shape[4]):
                acc += V[a, x, X, b, h, H] * S[b, u, U, c] * T[u, y, h, g, p] * np.conj(B[U, Y, H, G, p])
            ref[a, x, X, y, Y, c, g, G] = acc
    assert np.allclose(A, ref, rtol=1e-13, atol=1e-14)


@pytest.mark.parametrize("complex_", [False, True])
def test_rsvd_exact_regime_equals_definition(complex_):
    """k = min(rows, cols): the randomized SVD reproduces A and its spectrum."""
    rng = np.random.default_rng(3)
    op = zipup_operator(*_zip_inputs(rng, 2, 2, 2, 2, 2, 2, 2, 1, 2, complex_))
    A = op.explicit()
    kmax = min(op.n_rows, op.n_cols)
    om = sketch(11, 1, op.n_cols, kmax)
    U, s, Vh = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, kmax, 1, om)
    assert np.allclose((U * s) @ Vh, A, atol=1e-13 * np.abs(A).max() * 10)
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, s_ref[:kmax], atol=1e-13 * s_ref[0])
    assert np.allclose(U.conj().T @ U, np.eye(kmax), atol=1e-13)


def test_rsvd_low_rank_recovered_exactly():
    """rank(A) <= k: range(A Omega) = range(A), so the result is exact."""
    rng = np.random.default_rng(4)
    # carry with inner dims b*h*H = 1*2*2 = 4 limits the rank to 4
    op = zipup_operator(*_zip_inputs(rng, 4, 3, 1, 2, 2, 3, 3, 2, 2, False))
    A = op.explicit()
    s_ref = np.linalg.svd(A, compute_uv=False)
    assert s_ref[4] < 1e-13 * s_ref[0]
    om = sketch(5, 9, op.n_cols, 6)
    U, s, Vh = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, 4, 0, om)
    assert np.allclose((U * s) @ Vh, A, atol=1e-12 * s_ref[0])
    assert np.allclose(s, s_ref[:4], rtol=1e-12)


def test_rsvd_basis_invariance(monkeypatch):
    """The output depends only on the ranges of the sketches: replacing the
    orthonormal basis by a rotated one changes nothing but rounding."""
    rng = np.random.default_rng(5)
    op = zipup_operator(*_zip_inputs(rng, 3, 2, 3, 2, 2, 3, 2, 2, 2, True))
    om = sketch(3, 2, op.n_cols, 10)
    U0, s0, V0 = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, 6, 2, om)
    orig = rsvd.orthogonalize

    def rotated(Y):
        Q = orig(Y)
        Z = np.linalg.qr(rng.standard_normal((Q.shape[1],) * 2)
                         + 1j * rng.standard_normal((Q.shape[1],) * 2))[0]
        return Q @ Z

    monkeypatch.setattr(rsvd, "orthogonalize", rotated)
    U1, s1, V1 = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, 6, 2, om)
    assert np.allclose(s0, s1, rtol=1e-11)
    assert np.allclose((U0 * s0) @ V0, (U1 * s1) @ V1, atol=1e-11 * s0[0])


@pytest.mark.parametrize("complex_", [False, True])
def test_gram_eigh_orthogonalization(complex_):
    """Alg. 5 against what it must produce: Q an isometry, A = Q R, R^* R the
    Gram matrix, range(Q) = range(A) (same projector as a Householder QR)."""
    rng = np.random.default_rng(11)
    A = rng.standard_normal((300, 12))
    if complex_:
        A = A + 1j * rng.standard_normal((300, 12))
    Q, R = rsvd.orthogonalize_gram_eigh(A)
    assert np.max(np.abs(Q.conj().T @ Q - np.eye(12))) < 1e-13
    assert np.max(np.abs(Q @ R - A)) < 1e-13 * np.max(np.abs(A))
    assert np.max(np.abs(R.conj().T @ R - A.conj().T @ A)) < 1e-12 * np.linalg.norm(A, 2) ** 2
    Qh = np.linalg.qr(A)[0]
    assert np.max(np.abs(Q @ Q.conj().T - Qh @ Qh.conj().T)) < 1e-13


def test_gram_eigh_orthogonal_columns():
    """Special case: A with mutually orthogonal columns of distinct norms.  G
    is diagonal, so Q is A with its columns normalized (up to a sign per
    column) and R holds the norms."""
    rng = np.random.default_rng(2)
    Qh = np.linalg.qr(rng.standard_normal((40, 5)))[0]
    norms = np.array([5.0, 0.5, 3.0, 2.0, 1.0])
    A = Qh * norms
    Q, R = rsvd.orthogonalize_gram_eigh(A)
    order = np.argsort(norms)  # eigh sorts ascending
    for j, c in enumerate(order):
        assert abs(abs(Q[:, j] @ Qh[:, c]) - 1.0) < 1e-13
        assert abs(np.linalg.norm(R[j]) - norms[c]) < 1e-13 * norms.max()


def test_rsvd_gram_eigh_equals_householder(monkeypatch):
    """Alg. 4 with Alg. 5 as its orthogonalization gives the same truncated SVD
    as with Householder QR (the result depends on the ranges only)."""
    rng = np.random.default_rng(7)
    op = zipup_operator(*_zip_inputs(rng, 3, 2, 3, 2, 2, 3, 2, 2, 2, True))
    om = sketch(4, 1, op.n_cols, 10)
    U0, s0, V0 = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, 6, 1, om)
    monkeypatch.setattr(rsvd, "orthogonalize", lambda Y: rsvd.orthogonalize_gram_eigh(Y)[0])
    U1, s1, V1 = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, 6, 1, om)
    assert np.allclose(s0, s1, rtol=1e-10)
    assert np.allclose((U0 * s0) @ V0, (U1 * s1) @ V1, atol=1e-10 * s0[0])


def test_rsvd_near_optimal_on_pair_network():
    """Halko-type bound: with oversampling and power iterations the error is
    close to the optimal rank-m error (soft check, reported ratio <= 1.5)."""
    Bl, Br, T1, T2 = synth.pair_instance(m=6, D=2, d=2, seed=0, instance=0)
    op = pair_operator(Bl, Br, T1, T2)
    A = op.explicit()
    m, k = 6, 10
    om = sketch(0, 1, op.n_cols, k)
    U, s, Vh = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, m, 2, om)
    s_ref = np.linalg.svd(A, compute_uv=False)
    opt = np.sqrt(np.sum(s_ref[m:] ** 2))
    err = np.linalg.norm(A - (U * s) @ Vh)
    assert opt <= err <= 1.5 * opt
    assert np.all(s <= s_ref[:m] * (1 + 1e-12))  # Ritz values never exceed the true ones


def test_fix_gauge_canonical_and_product_invariant():
    rng = np.random.default_rng(8)
    U = np.linalg.qr(rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4)))[0]
    s = np.array([3.0, 2.0, 1.0, 0.5])
    Vh = np.linalg.qr(rng.standard_normal((7, 4)) + 1j * rng.standard_normal((7, 4)))[0].T.conj()
    U2, s2, V2 = rsvd.fix_gauge(U, s, Vh)
    assert np.allclose((U2 * s2) @ V2, (U * s) @ Vh, atol=1e-14)
    w = rsvd.gauge_vector(9)
    assert np.array_equal(w, sketch(0, 0, 9, 1)[:, 0])
    for i in range(4):
        z = w @ U2[:, i]
        assert z.real > 0 and abs(z.imag) < 1e-14
    # idempotent, and any column phase change is undone
    U3, _, V3 = rsvd.fix_gauge(U2 * np.exp(1j * np.arange(4)), s2, V2 * np.exp(-1j * np.arange(4))[:, None])
    assert np.allclose(U3, U2, atol=1e-14) and np.allclose(V3, V2, atol=1e-14)


def _explicit_power_reference(A, omega, m, q):
    """Alg. 4 (Sec. IV-A) by its definition rather than its steps: after q
    power iterations the sketch spans range((A A^*)^q A Omega), and the result
    is the best rank-m' approximation of A within that subspace, P (P^* A)_m'.
    The power is applied to the raw sketch without intermediate
    orthogonalization, the basis comes from an SVD instead of a QR, and the
    projected matrix P^* A is formed explicitly."""
    Y = A @ omega
    for _ in range(q):
        Y = A @ (A.conj().T @ Y)
    P = np.linalg.svd(Y, full_matrices=False)[0]
    W, s, Vh = np.linalg.svd(P.conj().T @ A, full_matrices=False)
    mp = min(m, omega.shape[1])
    return P @ W[:, :mp], s[:mp], Vh[:mp]


@pytest.mark.parametrize("complex_", [False, True])
def test_rsvd_power_iterations_match_explicit_krylov_power(complex_):
    """Pins the power loop: for q = 0..3 the randomized SVD equals the best
    rank-m' approximation of A inside range((A A^*)^q A Omega), computed from
    the explicit matrix power.  A gently decaying spectrum keeps the explicit
    power well conditioned (its columns span 0.9^(2q+1) decades at most) while
    the tail beyond k is large enough that every q gives a different answer,
    so a dropped or miscounted iteration fails."""
    rng = np.random.default_rng(21)
    n_rows, n_cols, k, m = 60, 50, 8, 5
    Ul = np.linalg.qr(_rand((n_rows, n_cols), rng, complex_))[0]
    Vr = np.linalg.qr(_rand((n_cols, n_cols), rng, complex_))[0]
    sv = 0.9 ** np.arange(n_cols)
    A = (Ul * sv) @ Vr.conj().T
    om = sketch(4, 2, n_cols, k)
    prods = []
    for q in range(4):
        U, s, Vh = rsvd.randomized_svd(lambda X: A @ X, lambda Y: A.conj().T @ Y,
                                       n_rows, n_cols, m, q, om)
        Ur, sr, Vhr = _explicit_power_reference(A, om, m, q)
        assert np.allclose(s, sr, rtol=0, atol=1e-11 * sv[0])
        prod = (U * s) @ Vh
        assert np.allclose(prod, (Ur * sr) @ Vhr, rtol=0, atol=1e-11 * sv[0])
        prods.append(prod)
    # each extra iteration changes the result far above the 1e-11 tolerance
    for q in range(3):
        assert np.abs(prods[q + 1] - prods[q]).max() > 1e-6 * sv[0]


def test_rsvd_error_ratio_per_power_iteration():
    """Halko et al.'s bound (cited in Sec. IV-A) tightens geometrically with q:
    on a pair network whose spectrum decays slowly the ratio of the error to
    the optimal rank-m error must fall into a distinct band for each q
    (q = 0 about 1.2, then within 1e-3, 1e-5, 1e-7 of the optimum)."""
    Bl, Br, T1, T2 = synth.pair_instance(m=6, D=2, d=2, seed=0, instance=0)
    op = pair_operator(Bl, Br, T1, T2)
    A = op.explicit()
    m, k = 6, 10
    om = sketch(0, 1, op.n_cols, k)
    s_ref = np.linalg.svd(A, compute_uv=False)
    opt = np.sqrt(np.sum(s_ref[m:] ** 2))
    ratio = []
    for q in range(4):
        U, s, Vh = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, m, q, om)
        ratio.append(np.linalg.norm(A - (U * s) @ Vh) / opt)
    assert ratio[0] > 1.1
    assert 1 + 1e-5 < ratio[1] <= 1.001
    assert 1 + 1e-8 < ratio[2] <= 1 + 1e-5
    assert 1 <= ratio[3] <= 1 + 1e-7
