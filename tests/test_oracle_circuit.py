"""Pins of the oracle's gate-list runner (oracle.ite.run_circuit): one-site
gates (Eq. 3), two-site gates on any two sites by SWAP chains (Sec. II-C),
checked against the state vector with bonds large enough to be lossless."""
import numpy as np
import pytest

import synth
from oracle import ite, statevector as sv


def _rand_gate(rng, shape):
    return rng.standard_normal(shape)


def _sv_circuit(psi, ops, gates2, gates1, ncol):
    for op in ops:
        if op[0] == 1:
            (i, j), g = op[1], op[2]
            psi = sv.apply_one_site(psi, gates1[g], i * ncol + j)
        else:
            (i1, j1), (i2, j2), g = op[1], op[2], op[3]
            psi = sv.apply_two_site(psi, gates2[g], i1 * ncol + j1, i2 * ncol + j2)
    return psi


def test_swap_gate_exchanges_sites():
    rng = np.random.default_rng(0)
    psi = rng.standard_normal((2, 2, 2))
    out = sv.apply_two_site(psi, ite.swap_gate(2), 0, 2)
    assert np.array_equal(out, psi.transpose(2, 1, 0))


@pytest.mark.parametrize("a,b", [((1, 1), (2, 2)), ((0, 0), (0, 3)), ((2, 0), (0, 3)), ((1, 2), (2, 1)),
                                 ((0, 1), (0, 0)), ((2, 3), (0, 0))])
def test_swap_path_steps_are_neighbours_and_end_adjacent(a, b):
    path = ite.swap_path(a, b)
    assert path[0] == b and a not in path
    for p, q in zip(path[:-1], path[1:]):
        assert abs(p[0] - q[0]) + abs(p[1] - q[1]) == 1
    assert abs(path[-1][0] - a[0]) + abs(path[-1][1] - a[1]) == 1


def test_circuit_lossless_equals_state_vector():
    """Random one-site and two-site gates on neighbours, diagonals and distant
    pairs of a 3 x 3 lattice (both orders of the sites), bonds uncapped."""
    rng = np.random.default_rng(1)
    peps = synth.product_state_peps(3, 3, seed=2)
    gates2 = [_rand_gate(rng, (2, 2, 2, 2)) for _ in range(3)]
    gates1 = [_rand_gate(rng, (2, 2)) for _ in range(2)]
    ops = [(1, (0, 0), 0), (2, (0, 0), (0, 1), 0), (2, (1, 1), (2, 2), 1), (2, (2, 1), (1, 2), 2),
           (1, (1, 1), 1), (2, (0, 2), (2, 0), 0), (2, (1, 0), (0, 0), 1)]
    out, spectra = ite.run_circuit(peps, ops, gates2, gates1, Dmax=64)
    ref = _sv_circuit(sv.peps_to_statevector(peps), ops, gates2, gates1, 3)
    got = sv.peps_to_statevector(out)
    # every QR-SVD update normalises its kept spectrum: compare directions
    ov = abs(np.vdot(got, ref)) / (np.linalg.norm(got) * np.linalg.norm(ref))
    assert abs(ov - 1) < 1e-12
    assert np.allclose(got / np.linalg.norm(got), ref / np.linalg.norm(ref) * np.sign(np.vdot(ref, got).real),
                       atol=1e-12)
    assert len(spectra) == 1 + 3 + 3 + 7 + 1   # SWAP chains of 0, 1, 1, 3 and 0 steps each way


def test_circuit_truncation_is_the_bond_cap():
    """With a cap, no bond exceeds it and the result differs from the lossless one."""
    rng = np.random.default_rng(3)
    peps = synth.random_peps(3, 3, 2, seed=4)
    gates2 = [_rand_gate(rng, (2, 2, 2, 2))]
    ops = [(2, (0, 0), (2, 2), 0), (2, (0, 2), (2, 0), 0)]
    out, _ = ite.run_circuit(peps, ops, gates2, [], Dmax=2)
    assert max(max(t.shape[:4]) for row in out for t in row) <= 2
