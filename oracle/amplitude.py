"""Amplitudes <i|psi> of a PEPS by the boundary-MPS contraction of a one-layer
network (test infrastructure: a plain NumPy statement of what the library's
amplitude computes; only the tests, the smoke check and the bench's CPU
baseline use it).

Fixing every physical leg to the basis state's bit turns the state into a
one-layer network of [u, d, l, r] slices (the amplitude network of Sec. III,
one layer fewer than the <psi|psi> network of the IBMPS).  It is contracted
from the top with the same steps as the two-layer norm (Alg. 2 with the
zip-up ApproxApply of Alg. 3):

* row 1 is the exact boundary: the slice of column j read as [l, d, r], each
  divided by its Frobenius norm;
* rows 2 .. n-1 are absorbed by the zip-up, left to right on the 1st, 3rd, ...
  absorbed row and right to left on the others.  The first column's carry
  C[a, x, b, h] = sum_u S[a, u, b] A[u, x, 1, h] is exact (and normalised);
  every later column is one randomized einsumsvd (Alg. 4, canonical phase as
  in rsvd.fix_gauge) of the implicit matrix with rows (a, x) and columns
  (y, c, g) of the network C[a,x,b,h] S[b,u,c] A[u,y,h,g]: U becomes the
  finished boundary tensor [a, x, m'] and (Sigma / sigma_1) V^* the next carry
  [m', y, c, g].  With explicit=True (BMPS, Sec. III-B) the matrix is formed
  and its truncated SVD taken by definition (rsvd.truncated_svd), with the
  same canonical phase;
* row n is contracted exactly, column by column, normalising the running
  vector.

The sketch of the einsumsvd that absorbs lattice column j of row i has stream
id 1 + (i * ncol + j) (the top-down pass); its column index runs over
(y, c, g) row-major, then the sketch column.  The logarithms of every
normalisation factor and every sigma_1 are summed, so that
<i|psi> = phase * exp(log_abs).  A slice that is exactly zero makes the
amplitude exactly zero: (log_abs, phase) = (-inf, 0).  Site tensors are not
rescaled first (the rescalings above keep every intermediate in range).
"""
import numpy as np

from .rsvd import fix_gauge, randomized_svd, sketch_width, truncated_svd
from .sketch import sketch, stream_id

L2R, R2L = 0, 1


def sliced_layer(ket, bits):
    """The one-layer network of <bits|psi>: site [u,d,l,r,p] -> [u,d,l,r] at p = bit
    (bits row-major over the sites)."""
    ncol = len(ket[0])
    return [[T[..., int(bits[i * ncol + j])] for j, T in enumerate(row)] for i, row in enumerate(ket)]


def _mirror_site(A):
    return A.transpose(0, 1, 3, 2)      # [u,d,l,r] -> [u,d,r,l]


def _mirror_bnd(S):
    return S.transpose(2, 1, 0)         # [l,x,r] -> [r,x,l]


def first_row(row):
    """Exact row-1 boundary [l, d, r] (u = 1), each tensor normalised."""
    out, log_scale = [], 0.0
    for A in row:
        S = A[0].transpose(1, 0, 2)      # [d,l,r] -> [l,d,r]
        nrm = np.linalg.norm(S)
        out.append(S / nrm)
        log_scale += np.log(nrm)
    return out, log_scale


def zipup_l2r(bnd, row, m, p, q, seed, sids, explicit=False):
    """Alg. 3 left to right on the one-layer network.  Returns (new boundary,
    log scale added); the boundary legs [a, x, b] are [left, down, right]."""
    n = len(row)
    C = np.einsum("auc,uyhg->aycg", bnd[0], row[0])   # h = 1 at the left edge
    nrm = np.linalg.norm(C)
    C = C / nrm
    log_scale = np.log(nrm)
    out = []
    for j in range(1, n):
        S, A = bnd[j], row[j]
        a, x, _, _ = C.shape
        _, y, _, g = A.shape
        c = S.shape[2]
        rows, cols = a * x, y * c * g

        def apply(X, C=C, S=S, A=A):
            X = X.reshape(y, c, g, -1)
            return np.einsum("axbh,buc,uyhg,ycgk->axk", C, S, A, X, optimize=True).reshape(rows, -1)

        def apply_adj(Y, C=C, S=S, A=A):
            Y = Y.reshape(a, x, -1)
            return np.einsum("axbh,buc,uyhg,axk->ycgk", C.conj(), S.conj(), A.conj(), Y,
                             optimize=True).reshape(cols, -1)

        if explicit:
            M = np.einsum("axbh,buc,uyhg->axycg", C, S, A, optimize=True).reshape(rows, cols)
            U, s, Vh = fix_gauge(*truncated_svd(M, m))
        else:
            k = sketch_width(m, p, rows, cols)
            omega = sketch(seed, sids[j], cols, k)
            U, s, Vh = randomized_svd(apply, apply_adj, rows, cols, m, q, omega)
        mp = s.shape[0]
        out.append(U.reshape(a, x, mp))
        C = ((s / s[0])[:, None] * Vh).reshape(mp, y, c, g)
        log_scale += np.log(s[0])
    mp, y, c, g = C.shape
    out.append(C.reshape(mp, y, c * g))
    return out, log_scale


def absorb_row(bnd, row, direction, m, p, q, seed, sids, explicit=False):
    """One zip-up in the given direction; sids[j] is the sketch stream of the
    einsumsvd that absorbs lattice column j."""
    if direction == L2R:
        return zipup_l2r(bnd, row, m, p, q, seed, sids, explicit)
    out, ls = zipup_l2r([_mirror_bnd(S) for S in reversed(bnd)], [_mirror_site(A) for A in reversed(row)],
                        m, p, q, seed, list(reversed(sids)), explicit)
    return [_mirror_bnd(S) for S in reversed(out)], ls


def last_row(bnd, row):
    """Exact contraction of the boundary with the last row (d = 1): (mantissa, log)."""
    E = np.ones((1, 1), dtype=np.result_type(bnd[0], row[0]))
    log_scale = 0.0
    for S, A in zip(bnd, row):
        E = np.einsum("bh,buc,uhg->cg", E, S, A[:, 0], optimize=True)
        nrm = np.linalg.norm(E)
        E = E / nrm
        log_scale += np.log(nrm)
    return E.reshape(()), log_scale


def amplitude(ket, bits, m, p, q, seed, explicit=False):
    """<bits|psi> by the one-layer boundary MPS (IBMPS, or BMPS with
    explicit=True, where p, q and seed are unused).  Returns (log_abs, phase)
    with <bits|psi> = phase * exp(log_abs); (-inf, 0) for an exactly zero slice."""
    layer = sliced_layer(ket, bits)
    if any(not np.any(A) for row in layer for A in row):
        return -np.inf, 0.0
    nrow, ncol = len(layer), len(layer[0])
    if nrow == 1:
        bnd, log_scale = [np.ones((1, 1, 1), dtype=layer[0][0].dtype)] * ncol, 0.0
    else:
        bnd, log_scale = first_row(layer[0])
        for t in range(1, nrow - 1):
            direction = L2R if t % 2 == 1 else R2L
            sids = [stream_id(0, nrow, ncol, t, j) for j in range(ncol)]
            bnd, ls = absorb_row(bnd, layer[t], direction, m, p, q, seed, sids, explicit)
            log_scale += ls
    v, ls = last_row(bnd, layer[nrow - 1])
    return log_scale + ls + np.log(abs(v)), v / abs(v)
