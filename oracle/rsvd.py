"""einsumsvd: the definition (explicit truncated SVD) and the method
(randomized SVD on an implicit operator, Alg. 4).

Sec. II-C defines einsumsvd as: contract a tensor network, matricize it by
splitting its open legs into a left and a right group, compute a low-rank
factorization (truncated SVD) and fold the factors back into two tensors
joined by one new leg.  Sec. IV-A replaces the explicit SVD by a randomized
SVD that only needs the products A @ X and A^* @ Y, which are evaluated as
tensor contractions without ever forming A.
"""
import numpy as np


def truncated_svd(A, m):
    """Definition: full LAPACK SVD of the explicit matrix, first m' = min(m, rows,
    cols) triplets, singular values non-increasing."""
    U, s, Vh = np.linalg.svd(A, full_matrices=False)
    mp = min(m, A.shape[0], A.shape[1])
    return U[:, :mp], s[:mp], Vh[:mp]


def sketch_width(m, p, n_rows, n_cols):
    """k = min(m + p, rows, cols): target rank plus oversampling, capped by the
    matrix shape (oversampling is not part of Alg. 4 itself, which sketches with
    exactly the target rank; it follows Halko et al., cited in Sec. IV-A)."""
    return min(m + p, n_rows, n_cols)


def orthogonalize(Y):
    """Orthonormal basis of range(Y) (Householder QR, reduced)."""
    return np.linalg.qr(Y, mode="reduced")[0]


def orthogonalize_gram_eigh(A):
    """Reshape-avoiding orthogonalization (Alg. 5, Sec. V): the Gram matrix
    G = A^* A, its eigendecomposition G = X Lambda X^*, R = Lambda^1/2 X^*,
    P = R^-1 = X Lambda^-1/2 and Q = A P.  Returns (Q, R) with A = Q R and Q
    an isometry (for full column rank A; it squares the condition number, so
    Q's orthogonality degrades like eps kappa(A)^2)."""
    G = A.conj().T @ A
    lam, X = np.linalg.eigh(G)
    lam = np.clip(lam, 0.0, None)
    R = np.sqrt(lam)[:, None] * X.conj().T
    P = X / np.sqrt(lam)[None, :]
    return A @ P, R


def randomized_svd(apply, apply_adj, n_rows, n_cols, m, q, omega):
    """Alg. 4 on an implicit operator A (n_rows x n_cols).

    apply(X)      -> A @ X        for X of shape (n_cols, k)
    apply_adj(Y)  -> A^* @ Y      for Y of shape (n_rows, k)
    omega         -> the sketch, shape (n_cols, k)
    q             -> number of power iterations (Alg. 4's iteration count)

    Returns U (n_rows x m'), s (m'), Vh (m' x n_cols) with m' = min(m, k).
    """
    k = omega.shape[1]
    assert omega.shape == (n_cols, k) and k <= min(n_rows, n_cols)
    P = orthogonalize(apply(omega))
    for _ in range(q):
        Q = orthogonalize(apply_adj(P))
        P = orthogonalize(apply(Q))
    B = apply_adj(P).conj().T            # P^* A, shape (k, n_cols)
    Ut, s, Vh = np.linalg.svd(B, full_matrices=False)
    mp = min(m, k)
    return fix_gauge(P @ Ut[:, :mp], s[:mp], Vh[:mp])


def gauge_vector(n):
    """The fixed vector w (length n) that defines the canonical phase: the
    counter-based uniform values of the sketch generator with seed 0 and
    stream 0, one column."""
    from .sketch import sketch
    return sketch(0, 0, n, 1)[:, 0]


def fix_gauge(U, s, Vh):
    """Canonical phase of each singular pair: the projection w . U[:, i] on the
    fixed vector w of gauge_vector is made real positive and V^*[i, :] is
    counter-rotated, so U diag(s) V^* is unchanged.  The paper leaves this
    phase free; it matters because a later randomized SVD sketches the
    resulting tensors in their index basis, so every implementation has to
    make the same choice to reproduce the same numbers.  (A rule based on the
    largest entry is not usable: in <psi|psi> networks the ket/bra symmetry
    produces entries of exactly equal magnitude.)"""
    U = U.copy()
    Vh = Vh.copy()
    w = gauge_vector(U.shape[0])
    for i in range(U.shape[1]):
        z = w @ U[:, i]
        if z != 0:
            ph = z / abs(z)
            U[:, i] *= np.conj(ph)
            Vh[i, :] *= ph
    return U, s, Vh

