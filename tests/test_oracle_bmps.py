"""Pins of the oracle's boundary-MPS contraction and brute-force state vectors."""
import numpy as np
import pytest

import synth
from oracle import bmps, statevector as sv


def _exact_m(D, ncol):
    return 10 ** 6  # far above any bond reached on the small lattices used here


def test_statevector_product_state_closed_form():
    peps = synth.product_state_peps(2, 3, seed=3, complex_=True)
    psi = sv.peps_to_statevector(peps)
    ref = np.ones(1)
    for row in peps:
        for t in row:
            ref = np.kron(ref, t.reshape(2))
    assert np.allclose(psi.ravel(), ref, atol=1e-15)


def test_statevector_two_sites_by_loops():
    rng = np.random.default_rng(0)
    T1 = rng.standard_normal((1, 1, 1, 3, 2))
    T2 = rng.standard_normal((1, 1, 3, 1, 2))
    psi = sv.peps_to_statevector([[T1, T2]])
    for p1 in range(2):
        for p2 in range(2):
            ref = sum(T1[0, 0, 0, h, p1] * T2[0, 0, h, 0, p2] for h in range(3))
            assert np.isclose(psi[p1, p2], ref, rtol=1e-14)


def test_statevector_vertical_bond_by_loops():
    rng = np.random.default_rng(1)
    T1 = rng.standard_normal((1, 3, 1, 1, 2))
    T2 = rng.standard_normal((3, 1, 1, 1, 2))
    psi = sv.peps_to_statevector([[T1], [T2]])
    ref = np.einsum("hp,hq->pq", T1[0, :, 0, 0, :], T2[:, 0, 0, 0, :])
    assert np.allclose(psi, ref, rtol=1e-14)


@pytest.mark.parametrize("complex_", [False, True])
@pytest.mark.parametrize("shape", [(2, 2), (3, 3), (3, 4), (4, 3)])
def test_bmps_exact_regime_equals_brute_force(shape, complex_):
    nrow, ncol = shape
    peps = synth.random_peps(nrow, ncol, D=2, seed=11, complex_=complex_)
    psi = sv.peps_to_statevector(peps)
    ref = np.log(np.vdot(psi, psi).real)
    for side in (bmps.TOP, bmps.BOTTOM):
        ln, ph = bmps.peps_norm(peps, m=10 ** 6, p=0, q=0, seed=1, side=side)
        assert abs(ln - ref) < 1e-11
        assert abs(ph - 1) < 1e-11


def test_bmps_c1_exact_regime_4x4():
    """4x4, D=2: the exact regime (m large) equals the 2^16-amplitude state vector."""
    peps = synth.random_peps(4, 4, D=2, seed=0)
    psi = sv.peps_to_statevector(peps)
    ref = np.log(np.vdot(psi, psi).real)
    ln, ph = bmps.peps_norm(peps, m=64, p=8, q=1, seed=0)
    assert abs(ln - ref) < 1e-10 and abs(ph - 1) < 1e-12


def test_bmps_c1_truncated_is_close():
    """m=4, p=4, q=1 truncates (exact bond 16); the error is small but not zero."""
    peps = synth.random_peps(4, 4, D=2, seed=0)
    psi = sv.peps_to_statevector(peps)
    ref = np.log(np.vdot(psi, psi).real)
    ln, ph = bmps.peps_norm(peps, m=4, p=4, q=1, seed=0)
    assert abs(ln - ref) < 0.1 and ph == pytest.approx(1.0)


def test_bmps_transposed_lattice_same_norm():
    peps = synth.random_peps(3, 4, D=2, seed=5, complex_=True)
    tr = [[peps[i][j].transpose(2, 3, 0, 1, 4) for i in range(3)] for j in range(4)]
    a = bmps.peps_norm(peps, m=10 ** 6, p=0, q=0, seed=0)[0]
    b = bmps.peps_norm(tr, m=10 ** 6, p=0, q=0, seed=0)[0]
    assert abs(a - b) < 1e-11


def test_bmps_product_state_norm_is_product():
    peps = synth.product_state_peps(4, 4, seed=2, complex_=True)
    scale = np.exp(np.random.default_rng(0).standard_normal((4, 4)))
    peps = [[peps[i][j] * scale[i, j] for j in range(4)] for i in range(4)]
    ln, ph = bmps.peps_norm(peps, m=4, p=2, q=1, seed=0)
    assert abs(ln - np.sum(2 * np.log(scale))) < 1e-12 and abs(ph - 1) < 1e-12


def test_bmps_tiny_scale_has_finite_log():
    peps = synth.random_peps(4, 4, D=2, seed=4)
    peps = [[t * 1e-200 for t in row] for row in peps]
    ln, _ = bmps.peps_norm(peps, m=64, p=0, q=0, seed=0)
    ref = bmps.peps_norm(synth.random_peps(4, 4, D=2, seed=4), m=64, p=0, q=0, seed=0)[0]
    assert np.isfinite(ln) and abs(ln - (ref + 16 * 2 * np.log(1e-200))) < 1e-9


def test_zipup_boundary_tensors_are_isometries():
    peps = synth.random_peps(4, 4, D=2, seed=6)
    envs, _ = bmps.boundary_pass(peps, peps, bmps.TOP, m=3, p=2, q=1, seed=0)
    # envs[1] was produced left to right: all but the last tensor are isometries
    for S in envs[1][:-1]:
        M = S.reshape(-1, S.shape[3])
        assert np.allclose(M.T @ M, np.eye(M.shape[1]), atol=1e-12)
    # envs[2] right to left: all but the first are isometries in the mirrored sense
    for S in envs[2][1:]:
        M = S.reshape(S.shape[0], -1)
        assert np.allclose(M @ M.T, np.eye(M.shape[0]), atol=1e-12)
