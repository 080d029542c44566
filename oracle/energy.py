"""Expectation values <psi|H|psi> / <psi|psi> of H = sum_t H_t (Eq. 5).

Cached (Sec. IV-B): two full boundary contractions, one from the top and one
from the bottom, store every intermediate boundary MPS.  A one-site or
horizontal two-site term on row i is then a contraction of a three-row strip
(top environment of row i-1, row i, bottom environment of row i+1); a
vertical term on rows i, i+1 uses a four-row strip.  Each term is the ratio
strip(term) / strip(identity) evaluated with the same left/right strip
environments, so all scale factors cancel.

Uncached: every term is an independent full boundary-MPS contraction of
<psi|H_t psi>, divided by <psi|psi>.  H_t psi is applied exactly: a one-site
operator acts on its site's physical leg; a two-site operator G is split into
d^2 products G = sum_{Q,q} G[:, Q, :, q] (x) |Q><q| (the elementary split: no
decomposition to compute), the first factor entering site 1 and the second
site 2, the pair index (Q, q) appended to their shared bond, which grows from
D to D d^2 (bond index (b, Q, q) row-major).  The bra psi is zero-padded to
the same bond dimensions, which leaves <psi|H_t psi> unchanged.

Trotter-Taylor (Eq. 6): <H> ~ (<psi|prod_j e^{tau H_j}|psi> / <psi|psi> - 1)
/ tau, with phi = prod_j G_j psi applied exactly gate by gate in the order
given (every bond a gate touches grows by d^2) and <psi|phi> contracted
against the zero-padded psi.

A term is (sites, op): sites a tuple of (i, j); op is [2,2] (out, in) for one
site or [2,2,2,2] (out1, out2, in1, in2) for two sites with site 1 left of /
above site 2: nearest neighbours, or (cached path only) diagonal neighbours
(i, j), (i + 1, j +- 1), the J2 pairs of Eq. 7, evaluated on the four-row
strip of their two rows over their two columns.
"""
import numpy as np

from .bmps import BOTTOM, TOP, boundary_pass, peps_norm


def operator_schmidt(op2, tol=1e-14):
    """op2[P1,P2,p1,p2] = sum_k A_k[P1,p1] B_k[P2,p2]."""
    d = op2.shape[0]
    M = op2.transpose(0, 2, 1, 3).reshape(d * d, d * d)
    U, s, Vh = np.linalg.svd(M)
    keep = s > tol * s[0]
    A = (U[:, keep] * s[keep]).T.reshape(-1, d, d)
    B = Vh[keep].reshape(-1, d, d)
    return list(zip(A, B))


def _trivial_env(ncol, dtype):
    return [np.ones((1, 1, 1, 1), dtype=dtype) for _ in range(ncol)]


# One column of a strip, one pairwise contraction per tensor (multi-operand
# einsum path searches can be orders of magnitude slower).
def _col3(L, Tp, T, O, B, Bt):
    TO = np.einsum("Pp,udlrp->udlrP", O, T)
    X = np.einsum("tlLb,tuUs->lLbuUs", L, Tp)
    X = np.einsum("lLbuUs,udlrP->LbUsdrP", X, TO)
    X = np.einsum("LbUsdrP,UDLRP->bsdrDR", X, B.conj())
    return np.einsum("bsdrDR,bdDc->srRc", X, Bt)


def _col4(L, Tp, T1, O1, B1, T2, O2, B2, Bt):
    T1O = np.einsum("Pp,uvlrp->uvlrP", O1, T1)
    T2O = np.einsum("Qq,vdmnq->vdmnQ", O2, T2)
    X = np.einsum("tlLmMb,tuUs->lLmMbuUs", L, Tp)
    X = np.einsum("lLmMbuUs,uvlrP->LmMbUsvrP", X, T1O)
    X = np.einsum("LmMbUsvrP,UVLRP->mMbsvrVR", X, B1.conj())
    X = np.einsum("mMbsvrVR,vdmnQ->MbsrVRdnQ", X, T2O)
    X = np.einsum("MbsrVRdnQ,VDMNQ->bsrRdnDN", X, B2.conj())
    return np.einsum("bsrRdnDN,bdDc->srRnNc", X, Bt)


def _mirror3(Tp, T, B, Bt):
    """The strip mirrored left-right: right environments are left ones of it."""
    return (Tp.transpose(3, 1, 2, 0), T.transpose(0, 1, 3, 2, 4), B.transpose(0, 1, 3, 2, 4),
            Bt.transpose(3, 1, 2, 0))


def _norm(x):
    n = np.linalg.norm(x)
    return x / n if n > 0 else x


def _row_terms(top, ket_row, bot, terms_here, d, dtype):
    """Three-row strip for one-site and horizontal terms of one lattice row."""
    n = len(ket_row)
    I = np.eye(d, dtype=dtype)
    Ls = [np.ones((1, 1, 1, 1), dtype=dtype)]
    for j in range(n):
        Ls.append(_norm(_col3(Ls[-1], top[j], ket_row[j], I, ket_row[j], bot[j])))
    # right environments by mirroring the transfer: contract from the right
    Rs = [np.ones((1, 1, 1, 1), dtype=dtype)]
    for j in reversed(range(n)):
        Tp, T, B, Bt = _mirror3(top[j], ket_row[j], ket_row[j], bot[j])
        Rs.append(_norm(_col3(Rs[-1], Tp, T, I, B, Bt)))
    Rs = Rs[::-1]  # Rs[j] = environment right of column j-1 (covers columns j..n-1)
    out = []
    for sites, op in terms_here:
        j = sites[0][1]
        if len(sites) == 1:
            num = np.vdot(Rs[j + 1].conj(), _col3(Ls[j], top[j], ket_row[j], op, ket_row[j], bot[j]))
            den = np.vdot(Rs[j + 1].conj(), _col3(Ls[j], top[j], ket_row[j], I, ket_row[j], bot[j]))
        else:
            num = 0.0
            for A, B in operator_schmidt(op):
                X = _col3(Ls[j], top[j], ket_row[j], A, ket_row[j], bot[j])
                X = _col3(X, top[j + 1], ket_row[j + 1], B, ket_row[j + 1], bot[j + 1])
                num = num + np.vdot(Rs[j + 2].conj(), X)
            X = _col3(Ls[j], top[j], ket_row[j], I, ket_row[j], bot[j])
            X = _col3(X, top[j + 1], ket_row[j + 1], I, ket_row[j + 1], bot[j + 1])
            den = np.vdot(Rs[j + 2].conj(), X)
        out.append((sites, num / den))
    return out


def _pair_terms(top, row1, row2, bot, terms_here, d, dtype):
    """Four-row strip for vertical terms between two lattice rows."""
    n = len(row1)
    I = np.eye(d, dtype=dtype)
    one = np.ones((1,) * 6, dtype=dtype)
    Ls = [one]
    for j in range(n):
        Ls.append(_norm(_col4(Ls[-1], top[j], row1[j], I, row1[j], row2[j], I, row2[j], bot[j])))
    Rs = [one]
    for j in reversed(range(n)):
        Tp, T1, _, Bt = _mirror3(top[j], row1[j], row1[j], bot[j])
        T2 = row2[j].transpose(0, 1, 3, 2, 4)
        Rs.append(_norm(_col4(Rs[-1], Tp, T1, I, T1, T2, I, T2, Bt)))
    Rs = Rs[::-1]
    out = []
    for sites, op in terms_here:
        j = sites[0][1]
        num = 0.0
        for A, B in operator_schmidt(op):
            X = _col4(Ls[j], top[j], row1[j], A, row1[j], row2[j], B, row2[j], bot[j])
            num = num + np.vdot(Rs[j + 1].conj(), X)
        X = _col4(Ls[j], top[j], row1[j], I, row1[j], row2[j], I, row2[j], bot[j])
        den = np.vdot(Rs[j + 1].conj(), X)
        out.append((sites, num / den))
    return out


def _diag_terms(top, row1, row2, bot, terms_here, d, dtype):
    """Four-row strip for diagonal terms between two lattice rows: site 1 at
    (i, j) and site 2 at (i + 1, j +- 1).  With op = sum_k A_k (x) B_k, A_k acts
    in site 1's column and B_k in site 2's, both columns between the left and
    right environments."""
    n = len(row1)
    I = np.eye(d, dtype=dtype)
    one = np.ones((1,) * 6, dtype=dtype)
    Ls = [one]
    for j in range(n):
        Ls.append(_norm(_col4(Ls[-1], top[j], row1[j], I, row1[j], row2[j], I, row2[j], bot[j])))
    Rs = [one]
    for j in reversed(range(n)):
        Tp, T1, _, Bt = _mirror3(top[j], row1[j], row1[j], bot[j])
        T2 = row2[j].transpose(0, 1, 3, 2, 4)
        Rs.append(_norm(_col4(Rs[-1], Tp, T1, I, T1, T2, I, T2, Bt)))
    Rs = Rs[::-1]

    def two_columns(a, ops_a, ops_b):
        X = _col4(Ls[a], top[a], row1[a], ops_a[0], row1[a], row2[a], ops_a[1], row2[a], bot[a])
        X = _col4(X, top[a + 1], row1[a + 1], ops_b[0], row1[a + 1], row2[a + 1], ops_b[1], row2[a + 1], bot[a + 1])
        return np.vdot(Rs[a + 2].conj(), X)

    out = []
    for sites, op in terms_here:
        (_, j1), (_, j2) = sites
        a = min(j1, j2)
        num = 0.0
        for A, B in operator_schmidt(op):
            if j1 < j2:   # site 1 in column a (upper row), site 2 in column a + 1 (lower row)
                num = num + two_columns(a, (A, I), (I, B))
            else:         # site 2 in column a (lower row), site 1 in column a + 1 (upper row)
                num = num + two_columns(a, (I, B), (A, I))
        den = two_columns(a, (I, I), (I, I))
        out.append((sites, num / den))
    return out


def peps_energy_cached(ket, terms, m, p, q, seed):
    """Returns (energy, per-term values in the order of ``terms``)."""
    nrow, ncol = len(ket), len(ket[0])
    d = ket[0][0].shape[4]
    dtype = np.result_type(*[t for row in ket for t in row], np.float64)
    top_envs, _ = boundary_pass(ket, ket, TOP, m, p, q, seed)
    bot_envs, _ = boundary_pass(ket, ket, BOTTOM, m, p, q, seed)
    triv = _trivial_env(ncol, dtype)

    def top_of(i):   # boundary above row i (rows 0..i-1 absorbed)
        return triv if i == 0 else top_envs[i - 1]

    def bot_of(i):   # boundary below row i (rows nrow-1..i+1 absorbed)
        return triv if i == nrow - 1 else bot_envs[nrow - 2 - i]

    values = {}
    for i in range(nrow):
        here = [(k, t) for k, t in enumerate(terms)
                if all(s[0] == i for s in t[0])]
        if here:
            res = _row_terms(top_of(i), ket[i], bot_of(i), [t for _, t in here], d, dtype)
            for (k, _), (_, v) in zip(here, res):
                values[k] = v
    for i in range(nrow - 1):
        here = [(k, t) for k, t in enumerate(terms)
                if len(t[0]) == 2 and t[0][0][0] == i and t[0][1][0] == i + 1 and t[0][0][1] == t[0][1][1]]
        if here:
            res = _pair_terms(top_of(i), ket[i], ket[i + 1], bot_of(i + 1),
                              [t for _, t in here], d, dtype)
            for (k, _), (_, v) in zip(here, res):
                values[k] = v
        diag = [(k, t) for k, t in enumerate(terms)
                if len(t[0]) == 2 and t[0][0][0] == i and t[0][1][0] == i + 1 and t[0][0][1] != t[0][1][1]]
        if diag:
            res = _diag_terms(top_of(i), ket[i], ket[i + 1], bot_of(i + 1), [t for _, t in diag], d, dtype)
            for (k, _), (_, v) in zip(diag, res):
                values[k] = v
    per_term = np.array([values[k] for k in range(len(terms))])
    return per_term.sum(), per_term


def _value(log_abs, phase):
    return phase * np.exp(log_abs)


def apply_one_site(T, O):
    """T'[u,d,l,r,P] = sum_p O[P,p] T[u,d,l,r,p]."""
    return np.einsum("Pp,udlrp->udlrP", O, T)


def apply_two_site_exact(S, T, G, vertical):
    """Exact application of G[P,Q,p,q] (out1, out2, in1, in2) to the neighbour
    sites S (left of / above) and T by the elementary split: S takes
    G[:, Q, :, q], T takes |Q><q|, and the pair (Q, q) joins their shared bond
    (new bond index (b, Q, q), row-major).  Returns (S', T')."""
    d = G.shape[0]
    E = np.zeros((d, d, d), dtype=G.dtype)          # E[Q, q, X] = delta(Q, X)
    for a in range(d):
        E[a, :, a] = 1.0
    if vertical:
        S2 = np.einsum("udlrp,PQpq->udQqlrP", S, G)
        T2 = np.einsum("udlrq,QqX->uQqdlrX", T, E)
        u, d1, l, r, P = S.shape
        S2 = S2.reshape(u, d1 * d * d, l, r, d)
        u2, dd, l2, r2, _ = T.shape
        T2 = T2.reshape(u2 * d * d, dd, l2, r2, d)
    else:
        S2 = np.einsum("udlrp,PQpq->udlrQqP", S, G)
        T2 = np.einsum("udlrq,QqX->udlQqrX", T, E)
        u, d1, l, r, P = S.shape
        S2 = S2.reshape(u, d1, l, r * d * d, d)
        u2, dd, l2, r2, _ = T.shape
        T2 = T2.reshape(u2, dd, l2 * d * d, r2, d)
    return S2, T2


def pad_site(T, shape):
    """T zero-padded to ``shape`` (every leg at least as long as T's)."""
    out = np.zeros(shape, dtype=T.dtype)
    out[tuple(slice(0, n) for n in T.shape)] = T
    return out


def _overlap_ratio(phi, ket, m, p, q, seed, ln, ph):
    """<ket|phi> / <ket|ket> with ket zero-padded to phi's shapes."""
    bra = [[pad_site(t, f.shape) for t, f in zip(rk, rf)] for rk, rf in zip(ket, phi)]
    l2, p2 = peps_norm(phi, m, p, q, seed, bra=bra)
    return _value(l2 - ln, p2 / ph)


def peps_energy_uncached(ket, terms, m, p, q, seed):
    """Eq. 5 term by term: each <psi|H_t psi> is its own boundary contraction of
    the exactly applied H_t psi against the zero-padded psi."""
    ln, ph = peps_norm(ket, m, p, q, seed)
    per_term = []
    for sites, op in terms:
        phi = [[t for t in row] for row in ket]
        if len(sites) == 1:
            (i, j), = sites
            phi[i][j] = apply_one_site(ket[i][j], op)
        else:
            (i1, j1), (i2, j2) = sites
            phi[i1][j1], phi[i2][j2] = apply_two_site_exact(ket[i1][j1], ket[i2][j2], op, i2 == i1 + 1)
        per_term.append(_overlap_ratio(phi, ket, m, p, q, seed, ln, ph))
    per_term = np.array(per_term)
    return per_term.sum(), per_term


def trotter_state(ket, gates):
    """phi = prod_j G_j psi, gates applied exactly in the order given; gates is
    a list of (((i1, j1), (i2, j2)), G[P,Q,p,q]) on nearest neighbours."""
    phi = [[t for t in row] for row in ket]
    for ((i1, j1), (i2, j2)), G in gates:
        phi[i1][j1], phi[i2][j2] = apply_two_site_exact(phi[i1][j1], phi[i2][j2], G, i2 == i1 + 1)
    return phi


def trotter_expectation(ket, gates, tau, m, p, q, seed):
    """Eq. 6: (<psi|phi> / <psi|psi> - 1) / tau with phi = trotter_state(ket,
    gates) (gates e^{tau H_j}).  Returns (estimate, <psi|phi> / <psi|psi>)."""
    ln, ph = peps_norm(ket, m, p, q, seed)
    ratio = _overlap_ratio(trotter_state(ket, gates), ket, m, p, q, seed, ln, ph)
    return (ratio - 1.0) / tau, ratio
