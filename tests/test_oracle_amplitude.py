"""Pins of the oracle's one-layer boundary-MPS amplitude against what does not
depend on it: the exact state vector (every einsumsvd lossless when the rank
covers the boundary), product-state closed forms, the completeness sum
sum_i |<i|psi>|^2 = <psi|psi>, and the zero-slice rule."""
import itertools

import numpy as np
import pytest

import synth
from oracle import amplitude as amp
from oracle import statevector as sv


def _value(log_abs, phase):
    return phase * np.exp(log_abs)


@pytest.mark.parametrize("shape,D", [((3, 3), 2), ((4, 3), 2), ((5, 2), 2), ((2, 4), 3), ((1, 4), 2), ((4, 1), 2)])
@pytest.mark.parametrize("cplx", [False, True])
def test_exact_regime_equals_state_vector(shape, D, cplx):
    """With m >= every boundary dimension each randomized SVD is exact (k = min(rows,
    cols)), so the zip-up reproduces the exact amplitude; lattices of 4 and 5 rows
    also sweep right to left."""
    nrow, ncol = shape
    ket = synth.random_peps(nrow, ncol, D, seed=nrow * 10 + ncol, complex_=cplx)
    psi = sv.peps_to_statevector(ket)
    rng = np.random.default_rng(1)
    for _ in range(4):
        bits = rng.integers(0, 2, nrow * ncol)
        la, ph = amp.amplitude(ket, bits, m=64, p=0, q=0, seed=3)
        ref = psi[tuple(bits)]
        assert abs(_value(la, ph) - ref) <= 1e-12 * np.abs(psi).max()
        assert abs(ph) == pytest.approx(1.0, abs=1e-14)


def test_product_state_closed_form():
    ket = synth.product_state_peps(3, 4, seed=5, complex_=True)
    for bits in ([0] * 12, [1] * 12, [0, 1] * 6, [1, 1, 0, 1, 0, 0, 1, 0, 1, 1, 0, 0]):
        want = np.prod([ket[i][j].ravel()[bits[i * 4 + j]] for i in range(3) for j in range(4)])
        la, ph = amp.amplitude(ket, bits, m=4, p=2, q=1, seed=0)
        assert abs(_value(la, ph) - want) <= 1e-13 * abs(want)


def test_completeness_matches_norm():
    """sum over all 2^N basis states of |<i|psi>|^2 equals <psi|psi> (exact regime)."""
    ket = synth.random_peps(2, 3, 2, seed=11, complex_=True)
    psi = sv.peps_to_statevector(ket)
    tot = 0.0
    for bits in itertools.product((0, 1), repeat=6):
        la, _ = amp.amplitude(ket, bits, m=16, p=0, q=0, seed=0)
        tot += np.exp(2 * la)
    assert tot == pytest.approx(np.vdot(psi, psi).real, rel=1e-12)


def test_zero_slice_is_exact_zero():
    ket = synth.random_peps(3, 3, 2, seed=2)
    ket[1][2] = ket[1][2].copy()
    ket[1][2][..., 1] = 0.0
    bits = [0] * 9
    bits[5] = 1
    assert amp.amplitude(ket, bits, m=4, p=2, q=1, seed=0) == (-np.inf, 0.0)
    bits[5] = 0
    la, _ = amp.amplitude(ket, bits, m=4, p=2, q=1, seed=0)
    assert np.isfinite(la)


def test_truncation_error_shrinks_with_rank():
    """In the truncating regime the error is the boundary truncation's: it falls
    to rounding once m covers the boundary (D = 3 on 4 x 4: bond dims up to 27)."""
    ket = synth.random_peps(4, 4, 3, seed=7)
    psi = sv.peps_to_statevector(ket)
    bits = np.random.default_rng(0).integers(0, 2, 16)
    ref = psi[tuple(bits)]
    errs = []
    for m in (2, 27):
        la, ph = amp.amplitude(ket, bits, m=m, p=4, q=2, seed=1)
        errs.append(abs(_value(la, ph) - ref) / np.abs(psi).max())
    assert errs[1] < 1e-12 < errs[0]


@pytest.mark.parametrize("cplx", [False, True])
def test_explicit_exact_regime_equals_state_vector(cplx):
    """BMPS (explicit matrix, dense truncated SVD) with m covering every
    boundary reproduces the exact amplitude."""
    ket = synth.random_peps(4, 3, 2, seed=21, complex_=cplx)
    psi = sv.peps_to_statevector(ket)
    rng = np.random.default_rng(5)
    for _ in range(3):
        bits = rng.integers(0, 2, 12)
        la, ph = amp.amplitude(ket, bits, m=64, p=0, q=0, seed=0, explicit=True)
        assert abs(_value(la, ph) - psi[tuple(bits)]) <= 1e-12 * np.abs(psi).max()


def test_explicit_is_the_limit_of_power_iterations():
    """With truncation, every BMPS step keeps the exact rank-m truncated SVD;
    the randomized SVD converges to it as the power iterations grow (the
    spectrum of each zip-up matrix has a gap at m), so IBMPS with many power
    iterations and oversampling reproduces BMPS."""
    ket = synth.random_peps(4, 4, 2, seed=8)
    bits = np.random.default_rng(2).integers(0, 2, 16)
    le, pe = amp.amplitude(ket, bits, m=3, p=0, q=0, seed=0, explicit=True)
    li, pi = amp.amplitude(ket, bits, m=3, p=5, q=60, seed=4)
    assert abs(le - li) < 1e-9 and abs(pe - pi) < 1e-9
    l0, _ = amp.amplitude(ket, bits, m=3, p=0, q=0, seed=4)
    assert abs(le - l0) > 1e-6   # without power iterations the two differ
