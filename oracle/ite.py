"""Imaginary-time evolution by TEBD with QR-SVD two-site updates.

Two-site update (Eq. 4, Alg. 1):
  1. QR-factor each site matricized as (other legs) x (shared bond, physical);
     when a site has no more rows than columns the factorization is skipped
     (Q = I, R = the matricized site), which changes nothing in exact
     arithmetic and avoids padding.
  2. Theta[(k1, i1'), (i2', k2)] = sum_{h, i1, i2} G[i1', i2', i1, i2]
                                     R1[k1, h, i1] R2[k2, h, i2]
     i.e. einsumsvd of (G, R1, R2), done with an explicit SVD because Theta
     is small.
  3. Keep the D' = min(D, rows, cols) largest singular values, normalise them
     to unit 2-norm, and put sqrt(s) into each side.
  4. Multiply the Q factors back.
A sweep applies exp(-tau H_b) to every bond, layer by layer: horizontal bonds
starting at even columns, then odd columns, then vertical bonds starting at
even rows, then odd rows (first-order Trotter splitting, Sec. II-D).
"""
import numpy as np

HORIZ, VERT = 0, 1


def _qr_or_identity(M):
    rows, cols = M.shape
    if rows <= cols:
        return np.eye(rows, dtype=M.dtype), M
    Q, R = np.linalg.qr(M, mode="reduced")
    return Q, R


def qr_svd_update(T1, T2, G, axis, Dmax):
    """Returns (T1', T2', kept singular values).  T1 is the left (HORIZ) or top
    (VERT) site; G[out1, out2, in1, in2]."""
    d = T1.shape[4]
    if axis == HORIZ:
        # T1 legs (u,d,l | r,p), T2 legs (u,d,r | l,p)
        o1 = T1.shape[:3]
        M1 = T1.reshape(-1, T1.shape[3] * d)
        T2p = T2.transpose(0, 1, 3, 2, 4)
        o2 = T2p.shape[:3]
        M2 = T2p.reshape(-1, T2.shape[2] * d)
        h = T1.shape[3]
    else:
        # T1 legs (u,l,r | d,p), T2 legs (d,l,r | u,p)
        T1p = T1.transpose(0, 2, 3, 1, 4)
        o1 = T1p.shape[:3]
        M1 = T1p.reshape(-1, T1.shape[1] * d)
        T2p = T2.transpose(1, 2, 3, 0, 4)
        o2 = T2p.shape[:3]
        M2 = T2p.reshape(-1, T2.shape[0] * d)
        h = T1.shape[1]
    Q1, R1 = _qr_or_identity(M1)
    Q2, R2 = _qr_or_identity(M2)
    k1, k2 = R1.shape[0], R2.shape[0]
    R1 = R1.reshape(k1, h, d)
    R2 = R2.reshape(k2, h, d)
    Theta = np.einsum("abcd,khc,lhd->kabl", G, R1, R2).reshape(k1 * d, d * k2)
    X, s, Yh = np.linalg.svd(Theta, full_matrices=False)
    Dn = min(Dmax, k1 * d, d * k2)
    s = s[:Dn] / np.linalg.norm(s[:Dn])
    sq = np.sqrt(s)
    R1n = (X[:, :Dn] * sq).reshape(k1, d * Dn)           # [k1, (i1', b)]
    R2n = (sq[:, None] * Yh[:Dn]).reshape(Dn, d, k2)     # [b, i2', k2]
    N1 = (Q1 @ R1n).reshape(o1 + (d, Dn))                # [o1..., p, b]
    N2 = (Q2 @ R2n.transpose(2, 0, 1).reshape(k2, Dn * d)).reshape(o2 + (Dn, d))  # [o2..., b, p]
    if axis == HORIZ:
        T1n = N1.transpose(0, 1, 2, 4, 3)                # [u,d,l,b,p]
        T2n = N2.transpose(0, 1, 3, 2, 4)                # [u,d,b,r,p]
    else:
        T1n = N1.transpose(0, 4, 1, 2, 3)                # [u,b,l,r,p]
        T2n = N2.transpose(3, 0, 1, 2, 4)                # [b,d,l,r,p]
    return np.ascontiguousarray(T1n), np.ascontiguousarray(T2n), s


def ite_sweep(peps, layers, gates, Dmax):
    """One TEBD sweep in place.  ``layers`` is the 4-layer bond list, ``gates``
    maps bond -> G.  Returns the kept singular values per bond in sweep order."""
    spectra = []
    for li, layer in enumerate(layers):
        axis = HORIZ if li < 2 else VERT
        for (s1, s2) in layer:
            (i1, j1), (i2, j2) = s1, s2
            T1n, T2n, s = qr_svd_update(peps[i1][j1], peps[i2][j2], gates[(s1, s2)], axis, Dmax)
            peps[i1][j1], peps[i2][j2] = T1n, T2n
            spectra.append(s)
    return spectra


def ite(peps, layers, gates, Dmax, n_sweeps):
    peps = [[t.copy() for t in row] for row in peps]
    spectra = None
    for _ in range(n_sweeps):
        spectra = ite_sweep(peps, layers, gates, Dmax)
    return peps, spectra


def swap_gate(d):
    """SWAP[P, Q, p, q] = delta(P, q) delta(Q, p)."""
    S = np.zeros((d, d, d, d))
    for a in range(d):
        for b in range(d):
            S[a, b, b, a] = 1.0
    return S


def apply_one_site(T, O):
    """Eq. 3: T'[u,d,l,r,P] = sum_p O[P,p] T[u,d,l,r,p]."""
    return np.einsum("Pp,udlrp->udlrP", O, T)


def _bond_update(peps, a, b, G, Dmax):
    """QR-SVD update of the neighbouring sites a and b with G acting on (a, b)
    in that order; the update itself takes the left / top site first, so G is
    transposed when b is left of or above a."""
    (ia, ja), (ib, jb) = a, b
    if (ia, ja + 1) == (ib, jb) or (ia + 1, ja) == (ib, jb):
        s1, s2, g = a, b, G
    else:
        assert (ib, jb + 1) == (ia, ja) or (ib + 1, jb) == (ia, ja), "sites are not neighbours"
        s1, s2, g = b, a, G.transpose(1, 0, 3, 2)
    axis = HORIZ if s1[0] == s2[0] else VERT
    T1n, T2n, s = qr_svd_update(peps[s1[0]][s1[1]], peps[s2[0]][s2[1]], g, axis, Dmax)
    peps[s1[0]][s1[1]], peps[s2[0]][s2[1]] = T1n, T2n
    return s


def swap_path(a, b):
    """Positions of site b's state on its way next to site a (Sec. II-C: a chain
    of SWAP gates on neighbouring sites): along b's row to a's column, then
    along that column, stopping at the first position adjacent to a."""
    (ia, ja), (ib, jb) = a, b
    path = [(ib, jb)]
    i, j = ib, jb
    while abs(i - ia) + abs(j - ja) != 1:
        if i != ia and j != ja:
            j += 1 if j < ja else -1
        elif i == ia:
            j += 1 if j < ja else -1
        else:
            i += 1 if i < ia else -1
        path.append((i, j))
    return path


def apply_gate_any(peps, a, b, G, Dmax):
    """A two-site gate on any two sites, in place: non-neighbours by moving b's
    state with SWAP gates (swap_path), applying G next to a, and moving it back
    (the SWAPs undone in reverse order).  Every update truncates to Dmax.
    Returns the kept singular values of every update in order."""
    d = G.shape[0]
    S = swap_gate(d)
    path = swap_path(a, b)
    spectra = []
    for p, q in zip(path[:-1], path[1:]):
        spectra.append(_bond_update(peps, p, q, S, Dmax))
    spectra.append(_bond_update(peps, a, path[-1], G, Dmax))
    for p, q in reversed(list(zip(path[:-1], path[1:]))):
        spectra.append(_bond_update(peps, p, q, S, Dmax))
    return spectra


def run_circuit(peps, ops, gates2, gates1, Dmax):
    """Applies a gate list in order: (2, a, b, g) the two-site gate gates2[g] on
    sites a, b (apply_gate_any), (1, a, g) the one-site gate gates1[g] on site a
    (Eq. 3).  Returns (new PEPS, kept singular values of every two-site update
    in order)."""
    peps = [[t.copy() for t in row] for row in peps]
    spectra = []
    for op in ops:
        if op[0] == 1:
            (i, j), g = op[1], op[2]
            peps[i][j] = apply_one_site(peps[i][j], gates1[g])
        else:
            spectra += apply_gate_any(peps, op[1], op[2], gates2[op[3]], Dmax)
    return peps, spectra
