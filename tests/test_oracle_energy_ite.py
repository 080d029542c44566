"""Pins of the oracle's expectation values (Eq. 5, Sec. IV-B) and of the
QR-SVD evolution (Alg. 1, Sec. II-D)."""
import numpy as np
import pytest

import synth
from oracle import energy, ite, statevector as sv

BIG_M = 10 ** 6  # exact regime on the small lattices used here


def tfi_terms(nrow, ncol, J=1.0, h=3.0):
    return [((s1, s2), Hb) for (s1, s2), Hb in synth.tfi_bond_hamiltonians(nrow, ncol, J, h).items()]


def heis_terms(nrow, ncol):
    Hb = synth.heisenberg_bond_hamiltonian()
    return [((s1, s2), Hb) for layer in synth.lattice_bonds(nrow, ncol) for (s1, s2) in layer]


def mixed_terms(nrow, ncol, seed=0):
    rng = np.random.default_rng(seed)
    terms = heis_terms(nrow, ncol)
    for i in range(nrow):
        for j in range(ncol):
            O = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2))
            terms.append((((i, j),), O + O.conj().T))
    return terms


def test_tfi_bond_split_sums_to_hamiltonian():
    """sum_b H_b equals -J sum ZZ - h sum X exactly (checked on a random state)."""
    nrow, ncol = 2, 3
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((2,) * 6) + 1j * rng.standard_normal((2,) * 6)
    e_split = sv.expectation(psi, tfi_terms(nrow, ncol, 1.0, 3.0), ncol)
    X, Z = synth.PAULI["X"], synth.PAULI["Z"]
    std = [((s1, s2), -np.einsum("ac,bd->abcd", Z, Z))
           for layer in synth.lattice_bonds(nrow, ncol) for (s1, s2) in layer]
    std += [(((i, j),), -3.0 * X) for i in range(nrow) for j in range(ncol)]
    assert np.isclose(e_split, sv.expectation(psi, std, ncol), rtol=1e-13)


def test_heisenberg_two_site_singlet():
    """XX+YY+ZZ has singlet eigenvalue -3 and triplet +1 (closed form)."""
    H = synth.heisenberg_bond_hamiltonian().reshape(4, 4)
    assert np.allclose(np.linalg.eigvalsh(H), [-3, 1, 1, 1], atol=1e-14)


def test_gate_is_exponential():
    Hb = synth.heisenberg_bond_hamiltonian()
    G = synth.bond_gate(Hb, 0.1).reshape(4, 4)
    # exp(-t H) for H with eigenvalues -3, 1: compare spectra, and the series
    assert np.allclose(np.sort(np.linalg.eigvalsh(G)), np.sort(np.exp(-0.1 * np.array([-3, 1, 1, 1]))))
    M = Hb.reshape(4, 4).real
    series = sum(np.linalg.matrix_power(-0.1 * M, n) / np.prod(np.arange(1, n + 1)) for n in range(25))
    assert np.allclose(G, series, atol=1e-14)


@pytest.mark.parametrize("shape", [(3, 3), (2, 4), (4, 2)])
def test_cached_energy_equals_brute_force(shape):
    nrow, ncol = shape
    peps = synth.random_peps(nrow, ncol, D=2, seed=3, complex_=True)
    terms = mixed_terms(nrow, ncol, seed=1)
    psi = sv.peps_to_statevector(peps)
    ref_terms = [sv.expectation(psi, [t], ncol) for t in terms]
    e, per = energy.peps_energy_cached(peps, terms, m=BIG_M, p=0, q=0, seed=0)
    assert np.allclose(per, ref_terms, rtol=1e-10, atol=1e-11)
    assert abs(e - sum(ref_terms)) < 1e-10 * max(1, abs(e))


def test_uncached_equals_cached_exact_regime():
    peps = synth.random_peps(3, 3, D=2, seed=8, complex_=True)
    terms = mixed_terms(3, 3, seed=2)
    e1, p1 = energy.peps_energy_cached(peps, terms, BIG_M, 0, 0, 0)
    e2, p2 = energy.peps_energy_uncached(peps, terms, BIG_M, 0, 0, 0)
    assert np.allclose(p1, p2, rtol=1e-10, atol=1e-11)


def test_cached_energy_converges_with_m():
    """Truncated environments approximate the exact energy and become exact once
    m reaches the exact boundary bond (16 for a 4x4 lattice with D=2)."""
    peps = synth.random_peps(4, 4, D=2, seed=9)
    terms = tfi_terms(4, 4)
    psi = sv.peps_to_statevector(peps)
    e_ref = sv.expectation(psi, terms, 4).real
    e12, _ = energy.peps_energy_cached(peps, terms, 12, 4, 1, 0)
    e16, _ = energy.peps_energy_cached(peps, terms, 16, 4, 1, 0)
    assert abs(e12 - e_ref) < 0.02 * abs(e_ref)
    assert abs(e16 - e_ref) < 1e-12


def test_product_state_energy_closed_form():
    peps = synth.product_state_peps(3, 4, seed=5, complex_=True)
    terms = mixed_terms(3, 4, seed=3)
    v = {(i, j): peps[i][j].reshape(2) for i in range(3) for j in range(4)}
    ref = 0
    for sites, op in terms:
        if len(sites) == 1:
            a = v[sites[0]]
            ref += np.vdot(a, op @ a)
        else:
            a, b = v[sites[0]], v[sites[1]]
            ref += np.einsum("P,Q,PQpq,p,q->", a.conj(), b.conj(), op, a, b)
    e, _ = energy.peps_energy_cached(peps, terms, 4, 2, 1, 0)
    assert abs(e - ref) < 1e-12


def _trotter_statevector(psi, layers, gates, ncol, n_sweeps):
    for _ in range(n_sweeps):
        for layer in layers:
            for (s1, s2) in layer:
                k, l = s1[0] * ncol + s1[1], s2[0] * ncol + s2[1]
                psi = sv.apply_two_site(psi, gates[(s1, s2)], k, l)
        psi = psi / np.linalg.norm(psi)
    return psi


@pytest.mark.parametrize("shape", [(2, 2), (2, 3), (3, 2)])
def test_ite_lossless_equals_statevector_trotter(shape):
    nrow, ncol = shape
    layers = synth.lattice_bonds(nrow, ncol)
    gates = {b: synth.bond_gate(H, 0.1) for b, H in synth.tfi_bond_hamiltonians(nrow, ncol, 1, 3).items()}
    peps0 = synth.product_state_peps(nrow, ncol, seed=1)
    peps, _ = ite.ite(peps0, layers, gates, Dmax=64, n_sweeps=3)
    psi = sv.peps_to_statevector(peps)
    ref = _trotter_statevector(sv.peps_to_statevector(peps0), layers, gates, ncol, 3)
    ov = abs(np.vdot(psi, ref)) / (np.linalg.norm(psi) * np.linalg.norm(ref))
    assert abs(ov - 1) < 1e-12


def test_ite_complex_gate_lossless():
    nrow, ncol = 2, 2
    layers = synth.lattice_bonds(nrow, ncol)
    rng = np.random.default_rng(4)
    Hr = rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4))
    gates = {b: synth.bond_gate((Hr + Hr.conj().T).reshape(2, 2, 2, 2), 0.2)
             for layer in layers for b in layer}
    peps0 = synth.random_peps(nrow, ncol, D=2, seed=2, complex_=True)
    peps, _ = ite.ite(peps0, layers, gates, Dmax=64, n_sweeps=2)
    psi = sv.peps_to_statevector(peps)
    ref = _trotter_statevector(sv.peps_to_statevector(peps0), layers, gates, ncol, 2)
    ov = abs(np.vdot(psi, ref)) / (np.linalg.norm(psi) * np.linalg.norm(ref))
    assert abs(ov - 1) < 1e-12


def test_ite_energy_variational_and_decreasing():
    """Energies of evolved states never go below the exact ground energy and
    decrease toward it (physics sanity)."""
    nrow, ncol = 2, 3
    layers = synth.lattice_bonds(nrow, ncol)
    terms = tfi_terms(nrow, ncol, 1.0, 3.0)
    gates = {b: synth.bond_gate(H, 0.05) for b, H in synth.tfi_bond_hamiltonians(nrow, ncol).items()}
    e0 = sv.ground_energy(terms, nrow * ncol, ncol)
    peps = synth.product_state_peps(nrow, ncol, seed=0)
    energies = []
    for _ in range(6):
        peps, _ = ite.ite(peps, layers, gates, Dmax=4, n_sweeps=10)
        energies.append(sv.expectation(sv.peps_to_statevector(peps), terms, ncol).real)
    assert all(e >= e0 - 1e-10 for e in energies)
    assert energies[-1] < energies[0]
    assert energies[-1] - e0 < 0.02 * abs(e0)


def test_ite_bond_growth_and_truncation():
    peps = synth.product_state_peps(4, 4, seed=0)
    layers = synth.lattice_bonds(4, 4)
    gates = {b: synth.bond_gate(H, 0.01) for b, H in synth.tfi_bond_hamiltonians(4, 4).items()}
    peps, spectra = ite.ite(peps, layers, gates, Dmax=3, n_sweeps=4)
    for row in peps:
        for T in row:
            assert max(T.shape[:4]) <= 3
    for s in spectra:
        assert np.isclose(np.linalg.norm(s), 1.0) and np.all(np.diff(s) <= 1e-15)


@pytest.mark.parametrize("vertical", [False, True])
def test_exact_two_site_application_matches_state_vector(vertical):
    """The elementary split applies G exactly: the state vector of the updated
    PEPS is G applied to the state vector (random complex G, both orientations)."""
    peps = synth.random_peps(3, 3, D=2, seed=4, complex_=True)
    rng = np.random.default_rng(6)
    G = rng.standard_normal((2, 2, 2, 2)) + 1j * rng.standard_normal((2, 2, 2, 2))
    (i1, j1), (i2, j2) = ((1, 1), (2, 1)) if vertical else ((1, 0), (1, 1))
    mod = [[t for t in row] for row in peps]
    mod[i1][j1], mod[i2][j2] = energy.apply_two_site_exact(peps[i1][j1], peps[i2][j2], G, vertical)
    assert mod[i1][j1].shape[1 if vertical else 3] == 8
    ref = sv.apply_two_site(sv.peps_to_statevector(peps), G, i1 * 3 + j1, i2 * 3 + j2)
    assert np.allclose(sv.peps_to_statevector(mod), ref, rtol=0, atol=1e-13 * np.abs(ref).max())


def test_uncached_energy_equals_brute_force():
    peps = synth.random_peps(2, 3, D=2, seed=12, complex_=True)
    terms = mixed_terms(2, 3, seed=5)
    psi = sv.peps_to_statevector(peps)
    ref = [sv.expectation(psi, [t], 3) for t in terms]
    _, per = energy.peps_energy_uncached(peps, terms, BIG_M, 0, 0, 0)
    assert np.allclose(per, ref, rtol=1e-10, atol=1e-11)


def _trotter_reference(peps, gates):
    psi = sv.peps_to_statevector(peps)
    phi = psi
    ncol = len(peps[0])
    for ((i1, j1), (i2, j2)), G in gates:
        phi = sv.apply_two_site(phi, G, i1 * ncol + j1, i2 * ncol + j2)
    return np.vdot(psi, phi) / np.vdot(psi, psi)


@pytest.mark.parametrize("shape", [(2, 3), (3, 2)])
def test_trotter_expectation_exact_regime(shape):
    """Eq. 6 with exact contractions equals the same Trotter product on the state
    vector: <psi| prod_j e^{tau H_j} |psi> / <psi|psi> at 1e-12."""
    nrow, ncol = shape
    peps = synth.random_peps(nrow, ncol, D=2, seed=nrow + 7 * ncol, complex_=True)
    tau = 0.05
    gates = [((s1, s2), synth.bond_gate(H, -tau)) for (s1, s2), H in
             synth.tfi_bond_hamiltonians(nrow, ncol, 1.0, 3.0).items()]
    est, ratio = energy.trotter_expectation(peps, gates, tau, BIG_M, 0, 0, 0)
    ref = _trotter_reference(peps, gates)
    assert abs(ratio - ref) < 1e-12 * abs(ref)
    assert abs(est - (ref - 1) / tau) < 1e-10


def test_trotter_expectation_is_first_order_in_tau():
    """The estimate approaches <H> linearly in tau: halving tau halves the error."""
    nrow, ncol = 2, 3
    peps = synth.random_peps(nrow, ncol, D=2, seed=3)
    hams = synth.tfi_bond_hamiltonians(nrow, ncol, 1.0, 3.0)
    exact = sv.expectation(sv.peps_to_statevector(peps), [((s1, s2), H) for (s1, s2), H in hams.items()],
                           ncol).real
    errs = []
    for tau in (0.02, 0.01, 0.005):
        gates = [((s1, s2), synth.bond_gate(H, -tau)) for (s1, s2), H in hams.items()]
        est, _ = energy.trotter_expectation(peps, gates, tau, BIG_M, 0, 0, 0)
        errs.append(abs(est.real - exact))
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3


@pytest.mark.parametrize("shape,cplx", [((3, 3), True), ((3, 4), False), ((4, 3), True)])
def test_cached_energy_with_diagonal_terms_equals_brute_force(shape, cplx):
    """J1-J2 terms (Eq. 7): nearest, both diagonal directions and fields, each
    term against the state vector in the exact regime."""
    nrow, ncol = shape
    peps = synth.random_peps(nrow, ncol, D=2, seed=nrow * ncol, complex_=cplx)
    terms = synth.j1j2_terms(nrow, ncol)
    psi = sv.peps_to_statevector(peps)
    ref = [sv.expectation(psi, [t], ncol) for t in terms]
    _, per = energy.peps_energy_cached(peps, terms, m=BIG_M, p=0, q=0, seed=0)
    assert np.allclose(per, ref, rtol=1e-10, atol=1e-11)
