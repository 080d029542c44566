"""Seeded synthetic inputs shared by the CPU oracle and the GPU library's tests/bench.

This module only *draws* inputs: random PEPS site tensors, random boundary-MPS
tensors, product states, Pauli matrices, the local Hamiltonian terms of the
models studied in the paper (transverse-field Ising as a special case of the
J1-J2 Hamiltonian, Eq. 7, and the Heisenberg model), and the two-site gate
``exp(-tau * H_bond)`` that the evolution algorithm takes as its input operator
(Alg. 1 requires the operator G as an input).  It contains none of the
contraction / factorization arithmetic of the method itself.

Conventions
-----------
* A site tensor has legs ``[u, d, l, r, p]`` (up, down, left, right, physical).
  Legs on the open boundary of the lattice have dimension 1.
* Lattices are lists of rows, each a list of site tensors, row-major.
* A two-site operator is stored as ``G[out1, out2, in1, in2]`` (the index order
  of the two-qubit gate in Sec. II-A, Eq. 2); site 1 is the left (horizontal
  bond) or the top (vertical bond) site.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "site_shape", "random_peps", "random_boundary_tensor", "product_state_peps",
    "pair_instance", "PAULI", "tfi_bond_hamiltonians", "heisenberg_bond_hamiltonian",
    "bond_gate", "lattice_bonds", "coordination", "diagonal_bonds", "j1j2_terms", "ry_gate", "CNOT",
    "vqe_ansatz_ops",
]


def site_shape(i, j, nrow, ncol, D, d):
    """Shape [u,d,l,r,p] of site (i, j) with open-boundary legs of dim 1."""
    return (1 if i == 0 else D, 1 if i == nrow - 1 else D,
            1 if j == 0 else D, 1 if j == ncol - 1 else D, d)


def _draw(rng, shape, complex_):
    if complex_:
        re = rng.standard_normal(shape)
        im = rng.standard_normal(shape)
        return re + 1j * im
    return rng.standard_normal(shape)


def random_peps(nrow, ncol, D, d=2, seed=0, complex_=False, normalize=True):
    """iid N(0,1) site tensors drawn in row-major site order from one generator.

    For complex tensors the real part is drawn before the imaginary part, site
    by site.  Each tensor is divided by its Frobenius norm when ``normalize``.
    """
    rng = np.random.default_rng(seed)
    rows = []
    for i in range(nrow):
        row = []
        for j in range(ncol):
            t = _draw(rng, site_shape(i, j, nrow, ncol, D, d), complex_)
            if normalize:
                t = t / np.linalg.norm(t)
            row.append(np.ascontiguousarray(t))
        rows.append(row)
    return rows


def random_boundary_tensor(mL, Dk, Db, mR, seed=0, complex_=False, normalize=True):
    """A boundary-MPS tensor [mL, D_ket, D_bra, mR], iid N(0,1), Frobenius 1."""
    rng = np.random.default_rng(seed)
    t = _draw(rng, (mL, Dk, Db, mR), complex_)
    if normalize:
        t = t / np.linalg.norm(t)
    return np.ascontiguousarray(t)


def pair_instance(m, D, d=2, seed=0, instance=0, complex_=False):
    """Inputs of one two-column einsumsvd instance (two adjacent boundary tensors
    Bl[a,u,U,b], Br[b,v,V,c] of shape [m,D,D,m] and two horizontally adjacent
    site tensors T1 [D,D,1,D,d], T2 [D,D,D,1,d] whose outer horizontal legs have
    dim 1), all iid N(0,1) and Frobenius-normalised, from generator (seed, instance).
    """
    rng = np.random.default_rng([seed, instance])
    out = []
    for shp in ((m, D, D, m), (m, D, D, m), (D, D, 1, D, d), (D, D, D, 1, d)):
        t = _draw(rng, shp, complex_)
        out.append(np.ascontiguousarray(t / np.linalg.norm(t)))
    return tuple(out)  # Bl, Br, T1, T2


def product_state_peps(nrow, ncol, d=2, seed=0, complex_=False):
    """Random product state: every site an N(0,1) d-vector, normalised, bond dim 1."""
    rng = np.random.default_rng(seed)
    rows = []
    for _ in range(nrow):
        row = []
        for _ in range(ncol):
            v = _draw(rng, (d,), complex_)
            v = v / np.linalg.norm(v)
            row.append(np.ascontiguousarray(v.reshape(1, 1, 1, 1, d)))
        rows.append(row)
    return rows


PAULI = {
    "I": np.eye(2, dtype=np.complex128),
    "X": np.array([[0, 1], [1, 0]], dtype=np.complex128),
    "Y": np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    "Z": np.array([[1, 0], [0, -1]], dtype=np.complex128),
}


def lattice_bonds(nrow, ncol):
    """Nearest-neighbour bonds grouped in the four layers of one sweep:
    horizontal-even, horizontal-odd, vertical-even, vertical-odd.  A bond is
    ((i1, j1), (i2, j2)) with site 1 left of / above site 2.  Within a layer
    no two bonds share a site."""
    he = [((i, j), (i, j + 1)) for i in range(nrow) for j in range(0, ncol - 1, 2)]
    ho = [((i, j), (i, j + 1)) for i in range(nrow) for j in range(1, ncol - 1, 2)]
    ve = [((i, j), (i + 1, j)) for i in range(0, nrow - 1, 2) for j in range(ncol)]
    vo = [((i, j), (i + 1, j)) for i in range(1, nrow - 1, 2) for j in range(ncol)]
    return [he, ho, ve, vo]


def coordination(nrow, ncol, i, j):
    """Number of nearest-neighbour bonds at site (i, j) on the open lattice."""
    return (i > 0) + (i < nrow - 1) + (j > 0) + (j < ncol - 1)


def _kron4(a, b):
    # 4x4 matrix of a (x) b reshaped to G[out1,out2,in1,in2]
    return np.einsum("ac,bd->abcd", a, b)


def tfi_bond_hamiltonians(nrow, ncol, J=1.0, h=3.0):
    """Transverse-field Ising, H = -J sum_<ij> Z_i Z_j - h sum_i X_i, written as a
    sum of bond terms: the field on a site is split evenly over its bonds, so
    summing the returned terms over all bonds gives H exactly.  Returns a dict
    bond -> H_b as [2,2,2,2] (out1,out2,in1,in2), complex128."""
    X, Z, I = PAULI["X"], PAULI["Z"], PAULI["I"]
    terms = {}
    for layer in lattice_bonds(nrow, ncol):
        for (s1, s2) in layer:
            z1 = coordination(nrow, ncol, *s1)
            z2 = coordination(nrow, ncol, *s2)
            Hb = -J * _kron4(Z, Z) - h * (_kron4(X, I) / z1 + _kron4(I, X) / z2)
            terms[(s1, s2)] = Hb
    return terms


def heisenberg_bond_hamiltonian(J=1.0):
    """Pauli-form Heisenberg bond term J (XX + YY + ZZ) as [2,2,2,2]."""
    X, Y, Z = PAULI["X"], PAULI["Y"], PAULI["Z"]
    return J * (_kron4(X, X) + _kron4(Y, Y) + _kron4(Z, Z))


def bond_gate(Hb, tau):
    """exp(-tau * H_b) for a Hermitian bond term, via its eigendecomposition.
    Returned as G[out1,out2,in1,in2]; real-valued Hamiltonians give a real gate
    (returned as float64 when the imaginary part is exactly zero)."""
    M = Hb.reshape(4, 4)
    if np.all(np.imag(M) == 0):
        M = np.real(M)
    w, V = np.linalg.eigh(M)
    G = (V * np.exp(-tau * w)) @ V.conj().T
    return np.ascontiguousarray(G.reshape(2, 2, 2, 2))


def diagonal_bonds(nrow, ncol):
    """Diagonally adjacent pairs ((k, l), (k+1, l+1)) and ((k, l), (k+1, l-1))."""
    down_right = [((i, j), (i + 1, j + 1)) for i in range(nrow - 1) for j in range(ncol - 1)]
    down_left = [((i, j), (i + 1, j - 1)) for i in range(nrow - 1) for j in range(1, ncol)]
    return down_right + down_left


def j1j2_terms(nrow, ncol, J1=(1.0, 1.0, 1.0), J2=(0.5, 0.5, 0.5), h=(0.2, 0.2, 0.2)):
    """The J1-J2 Heisenberg model in Pauli form (the paper's Eq. 7): J1 (x, y, z)
    couplings on nearest neighbours, J2 on diagonal neighbours, field h on every
    site.  Returns a list of (sites, op): two-site ops [2,2,2,2] (out1, out2,
    in1, in2) and one-site ops [2,2], complex128."""
    X, Y, Z = PAULI["X"], PAULI["Y"], PAULI["Z"]

    def coupling(J):
        return J[0] * _kron4(X, X) + J[1] * _kron4(Y, Y) + J[2] * _kron4(Z, Z)

    terms = [(b, coupling(J1)) for layer in lattice_bonds(nrow, ncol) for b in layer]
    terms += [(b, coupling(J2)) for b in diagonal_bonds(nrow, ncol)]
    terms += [(((i, j),), h[0] * X + h[1] * Y + h[2] * Z) for i in range(nrow) for j in range(ncol)]
    return terms


def ry_gate(theta):
    """R_y(theta) = exp(-i theta Y / 2) (a real rotation)."""
    c, s = np.cos(theta / 2), np.sin(theta / 2)
    return np.array([[c, -s], [s, c]])


# CNOT[P, Q, p, q] = delta(P, p) delta(Q, q xor p): site 1 controls site 2
CNOT = np.zeros((2, 2, 2, 2))
for _p in range(2):
    for _q in range(2):
        CNOT[_p, _q ^ _p, _p, _q] = 1.0


def vqe_ansatz_ops(nrow, ncol, n_layers):
    """The VQE ansatz circuit of the paper's Sec. VI-D as a gate list: each layer
    applies R_y to every qubit, then a CNOT to every nearest-neighbour pair (in
    the order of lattice_bonds).  Returns ops [(1, site, k) for the k-th R_y
    angle] + [(2, s1, s2, 0) for CNOT], with one angle per qubit and layer."""
    ops = []
    k = 0
    for _ in range(n_layers):
        for i in range(nrow):
            for j in range(ncol):
                ops.append((1, (i, j), k))
                k += 1
        for layer in lattice_bonds(nrow, ncol):
            for (s1, s2) in layer:
                ops.append((2, s1, s2, 0))
    return ops
