"""Boundary-MPS contraction of a two-layer PEPS network <bra|ket>.

* Row 1 of the network is the initial boundary MPS, kept exact (Alg. 2, first
  step).  Its bond is the ket bond times the bra bond.
* Rows 2 .. n-1 are absorbed one at a time by the zip-up ApproxApply (Alg. 3):
  the first column's carry is contracted exactly, and every later column runs
  one einsumsvd (randomized SVD on the implicit zip-up operator, Alg. 4) that
  finalizes the previous boundary tensor and hands a carry to the next column.
* The zip-up direction alternates from row to row (Sec. III-B: the factor that
  absorbs the singular values alternates between rows).  Here the singular
  values always go into the carry, so the finished tensors are isometries,
  and the alternation is realised by sweeping left-to-right on odd-numbered
  absorbed rows and right-to-left on even-numbered ones.
* Row n is contracted exactly (the last ApproxApply would be lossless: every
  one of its einsumsvds has at most m rows).

Scale: every exact row-1 tensor and every first-column carry is divided by its
Frobenius norm, and after every einsumsvd the singular values are divided by
the largest one; the logarithms of these factors are accumulated so that the
network value is exp(log_scale) * (contracted mantissa).

Leg conventions: site [u,d,l,r,p]; boundary tensor [mL, x_ket, X_bra, mR]
where x/X are the legs that connect to the next row to be absorbed.
"""
import numpy as np

from .network import zipup_operator
from .rsvd import randomized_svd, sketch_width
from .sketch import sketch, stream_id

L2R, R2L = 0, 1
TOP, BOTTOM = 0, 1


def mirror_lr_site(T):
    return T.transpose(0, 1, 3, 2, 4)


def mirror_ud_site(T):
    return T.transpose(1, 0, 2, 3, 4)


def mirror_lr_bnd(S):
    return S.transpose(3, 1, 2, 0)


def first_row_boundary(ket_row, bra_row):
    """Exact row-1 boundary S_j[(l,L), d, D, (r,R)] = sum_p T conj(B) with u = U = 1."""
    out, log_scale = [], 0.0
    for T, B in zip(ket_row, bra_row):
        S = np.einsum("udlrp,UDLRp->lLdDrR", T[:1], B[:1].conj())
        l, L, d, Dd, r, R = S.shape
        S = S.reshape(l * L, d, Dd, r * R)
        nrm = np.linalg.norm(S)
        out.append(S / nrm)
        log_scale += np.log(nrm)
    return out, log_scale


def zipup_row_l2r(bnd, ket_row, bra_row, m, p, q, seed, stream_ids):
    """Alg. 3 left to right.  Returns (new boundary tensors, log scale added,
    per-column singular values)."""
    n = len(ket_row)
    log_scale = 0.0
    V = np.einsum("buUc,uyhgp,UYHGp->byYcgG", bnd[0], ket_row[0], bra_row[0].conj())
    nrm = np.linalg.norm(V)
    V = V / nrm
    log_scale += np.log(nrm)
    out, spectra = [], []
    for j in range(1, n):
        op = zipup_operator(V, bnd[j], ket_row[j], bra_row[j])
        k = sketch_width(m, p, op.n_rows, op.n_cols)
        omega = sketch(seed, stream_ids[j], op.n_cols, k)
        U, s, Vh = randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, m, q, omega)
        mp = s.shape[0]
        a, x, X = op.rows_shape
        out.append(U.reshape(a, x, X, mp))
        spectra.append(s)
        V = ((s / s[0])[:, None] * Vh).reshape((mp,) + op.cols_shape)
        log_scale += np.log(s[0])
    a, y, Y, c, g, G = V.shape
    out.append(V.reshape(a, y, Y, c * g * G))
    return out, log_scale, spectra


def absorb_row(bnd, ket_row, bra_row, direction, m, p, q, seed, stream_ids):
    """One ApproxApply (Alg. 3) in the given direction.  ``stream_ids[j]`` is the
    sketch stream of the einsumsvd that absorbs lattice column j."""
    if direction == L2R:
        return zipup_row_l2r(bnd, ket_row, bra_row, m, p, q, seed, stream_ids)
    out, ls, spectra = zipup_row_l2r(
        [mirror_lr_bnd(S) for S in reversed(bnd)],
        [mirror_lr_site(T) for T in reversed(ket_row)],
        [mirror_lr_site(B) for B in reversed(bra_row)],
        m, p, q, seed, list(reversed(stream_ids)))
    return [mirror_lr_bnd(S) for S in reversed(out)], ls, spectra[::-1]


def contract_last_row(bnd, ket_row, bra_row):
    """Exact contraction of the boundary MPS with the last row (d = D = 1 legs).
    Returns (mantissa, log scale)."""
    E = np.ones((1, 1, 1), dtype=np.result_type(bnd[0], ket_row[0], bra_row[0]))
    log_scale = 0.0
    for S, T, B in zip(bnd, ket_row, bra_row):
        E = np.einsum("bhH,buUc,uyhgp,UYHGp->cgG", E, S, T[:, :1], B[:, :1].conj(), optimize=True)
        nrm = np.linalg.norm(E)
        if nrm > 0:
            E = E / nrm
            log_scale += np.log(nrm)
    return E.reshape(()), log_scale


def contract_boundary_chain(bnd):
    """Value of a boundary MPS whose x/X legs are all dim 1 (one-row lattice)."""
    E = np.ones((1,), dtype=bnd[0].dtype)
    log_scale = 0.0
    for S in bnd:
        E = E @ S[:, 0, 0, :]
        nrm = np.linalg.norm(E)
        E, log_scale = E / nrm, log_scale + np.log(nrm)
    return E.reshape(()), log_scale


def _oriented(ket, bra, side):
    if side == TOP:
        return ket, bra
    flip = lambda L: [[mirror_ud_site(T) for T in row] for row in reversed(L)]
    return flip(ket), flip(bra)


def boundary_pass(ket, bra, side, m, p, q, seed, upto=None):
    """Contract rows from one side, storing every intermediate boundary MPS.

    Returns (envs, logs) where envs[t] is the boundary after absorbing the first
    t+1 rows seen from ``side`` (t = 0 is the exact first row) and logs[t] its
    accumulated log scale.  ``upto`` bounds the number of rows absorbed
    (default: all but the last row)."""
    nrow, ncol = len(ket), len(ket[0])
    K, Bb = _oriented(ket, bra, side)
    upto = nrow - 1 if upto is None else upto
    bnd, log_scale = first_row_boundary(K[0], Bb[0])
    envs, logs = [bnd], [log_scale]
    for t in range(1, upto):
        orig_row = t if side == TOP else nrow - 1 - t
        direction = L2R if t % 2 == 1 else R2L
        sids = [stream_id(side, nrow, ncol, orig_row, j) for j in range(ncol)]
        bnd, ls, _ = absorb_row(bnd, K[t], Bb[t], direction, m, p, q, seed, sids)
        log_scale += ls
        envs.append(bnd)
        logs.append(log_scale)
    return envs, logs


def normalized_sites(layer):
    """Divide every site tensor by its Frobenius norm; returns (sites, sum of logs).
    Exact rescaling that keeps products of many tiny or huge tensors in range."""
    out, log_scale = [], 0.0
    for row in layer:
        new = []
        for T in row:
            mx = np.abs(T).max()          # two-step scaling: the sum of squares of
            T = T / mx                    # a tensor of 1e-200 entries underflows
            nrm = np.linalg.norm(T)
            new.append(T / nrm)
            log_scale += np.log(nrm) + np.log(mx)
        out.append(new)
    return out, log_scale


def peps_norm(ket, m, p, q, seed, bra=None, side=TOP):
    """<bra|ket> by boundary MPS (Alg. 2).  Returns (log|v|, phase) with
    v = phase * exp(log|v|); for bra = ket the value is the squared norm.
    Site tensors are first rescaled to unit norm (the scales go to the log)."""
    bra = ket if bra is None else bra
    ket, lk = normalized_sites(ket)
    bra, lb = normalized_sites(bra)
    ln, ph = _peps_norm(ket, bra, m, p, q, seed, side)
    return ln + lk + lb, ph


def _peps_norm(ket, bra, m, p, q, seed, side):
    nrow = len(ket)
    K, Bb = _oriented(ket, bra, side)
    if nrow == 1:
        bnd, ls = first_row_boundary(K[0], Bb[0])
        v, ls2 = contract_boundary_chain(bnd)
        return ls + ls2 + np.log(abs(v)), v / abs(v)
    envs, logs = boundary_pass(ket, bra, side, m, p, q, seed)
    v, ls = contract_last_row(envs[-1], K[nrow - 1], Bb[nrow - 1])
    return logs[-1] + ls + np.log(abs(v)), v / abs(v)
