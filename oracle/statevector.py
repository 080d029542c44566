"""Brute-force state vectors (Sec. II-A): the exact amplitude tensor of a small
PEPS, gate application by Eqs. 1-2, inner products, norms, energies and exact
diagonalisation.  Feasible up to ~22 sites.

Amplitudes are ordered by the physical indices of the sites in row-major
lattice order (site (i, j) is qubit i * ncol + j).
"""
import numpy as np


def peps_to_statevector(peps):
    """Contract every bond of the PEPS exactly; returns psi of shape (2,)*N."""
    nrow, ncol = len(peps), len(peps[0])
    d = peps[0][0].shape[4]
    # psi axes: [phys of all finished sites..., open down bonds of current frontier (ncol)]
    psi = np.ones((1,) * ncol, dtype=np.result_type(*[t for row in peps for t in row]))
    nphys = 0
    for i in range(nrow):
        # absorb row i column by column; carry a horizontal bond axis
        psi = psi[..., None]  # append left-bond axis (dim 1) at the end
        for j in range(ncol):
            T = peps[i][j]  # [u,d,l,r,p]
            # psi axes: [phys(nphys), down bonds of cols < j (j axes), up bonds of cols >= j
            #            (ncol - j axes), h]
            ax_up = nphys + j
            ax_h = psi.ndim - 1
            psi = np.tensordot(psi, T, axes=([ax_up, ax_h], [0, 2]))
            # new trailing axes: d, r, p ; move p to the physical block, d to position
            psi = np.moveaxis(psi, -1, nphys)           # p
            nphys += 1
            psi = np.moveaxis(psi, -2, nphys + j)       # d goes after previous downs
            # r is now last: the next h
        psi = psi[..., 0]  # right bond of the last column has dim 1
    psi = psi.reshape(psi.shape[:nphys])  # bottom down bonds are dim 1
    return psi


def apply_one_site(psi, g, k):
    """Eq. 1: t'_{..i_k..} = sum_j g[i_k, j] t_{..j..}."""
    out = np.tensordot(g, psi, axes=([1], [k]))
    return np.moveaxis(out, 0, k)


def apply_two_site(psi, g, k, l):
    """Eq. 2 with g[i_k, i_l, j_k, j_l]."""
    out = np.tensordot(g, psi, axes=([2, 3], [k, l]))
    return np.moveaxis(out, [0, 1], [k, l])


def inner(phi, psi):
    return np.vdot(phi.ravel(), psi.ravel())


def expectation(psi, terms, ncol):
    """<psi|H|psi>/<psi|psi> for H = sum of terms; a term is (sites, op) with
    sites a tuple of (i, j) and op [2,2] or [2,2,2,2]."""
    nrm = inner(psi, psi)
    e = 0.0
    for sites, op in terms:
        ks = [i * ncol + j for (i, j) in sites]
        if len(ks) == 1:
            phi = apply_one_site(psi, op, ks[0])
        else:
            phi = apply_two_site(psi, op, ks[0], ks[1])
        e = e + inner(psi, phi)
    return e / nrm


def hamiltonian_matrix(terms, nsites, ncol):
    """Dense-free sparse matrix of H (for exact diagonalisation)."""
    import scipy.sparse as sp
    dim = 2 ** nsites
    H = sp.csr_matrix((dim, dim), dtype=np.complex128)
    I2 = sp.identity(2, format="csr")
    for sites, op in terms:
        ks = [i * ncol + j for (i, j) in sites]
        if len(ks) == 1:
            mats = [I2] * nsites
            mats[ks[0]] = sp.csr_matrix(op)
            M = mats[0]
            for t in mats[1:]:
                M = sp.kron(M, t, format="csr")
        else:
            k, l = ks
            assert k < l
            opm = op.reshape(4, 4)
            # operator on qubits k..l with identities in between
            mid = l - k - 1
            blk = sp.kron(sp.identity(1), sp.csr_matrix(opm))
            if mid > 0:
                # apply by permutation-free construction: sum over op components
                o = op.reshape(2, 2, 2, 2)
                blk = None
                for a in range(2):
                    for b in range(2):
                        for c in range(2):
                            for dd in range(2):
                                v = o[a, b, c, dd]
                                if v == 0:
                                    continue
                                ea = sp.csr_matrix(([1.0], ([a], [c])), shape=(2, 2))
                                eb = sp.csr_matrix(([1.0], ([b], [dd])), shape=(2, 2))
                                t = sp.kron(sp.kron(ea, sp.identity(2 ** mid)), eb) * v
                                blk = t if blk is None else blk + t
            M = sp.kron(sp.identity(2 ** k), sp.kron(blk, sp.identity(2 ** (nsites - l - 1))),
                        format="csr")
        H = H + M
    return H


def ground_energy(terms, nsites, ncol):
    from scipy.sparse.linalg import eigsh
    H = hamiltonian_matrix(terms, nsites, ncol)
    w = eigsh(H, k=1, which="SA", return_eigenvectors=False)
    return float(np.real(w[0]))
