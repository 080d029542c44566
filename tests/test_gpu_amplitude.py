"""GPU parity of hpeps_peps_amplitude (one-layer boundary MPS) against the
oracle's amplitude on the same seeded lattices and sketch streams: truncating
regimes (every einsumsvd keeps m < its rank), both sweep directions, real and
complex sites, one-row and one-column lattices, the exact regime against the
state vector, the zero-slice rule and argument errors."""
import numpy as np
import pytest

import synth
from oracle import amplitude as amp
from oracle import statevector as sv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def dev_lattice(peps):
    return [[torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in row] for row in peps]


def _bits(n, seed):
    return [int(v) for v in np.random.default_rng(seed).integers(0, 2, n)]


# (nrow, ncol, D, m, p, q, complex): rows 4+ sweep right to left as well
CASES = [(3, 3, 2, 2, 2, 1, False), (4, 4, 3, 4, 2, 1, False), (5, 4, 2, 3, 1, 2, False),
         (6, 5, 3, 5, 3, 1, False), (4, 3, 3, 4, 2, 1, True), (5, 5, 2, 3, 2, 0, True),
         (1, 6, 3, 2, 1, 1, False), (6, 1, 3, 2, 1, 1, True), (2, 5, 4, 3, 2, 1, False)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:3])) + ("c" if c[6] else ""))
def test_amplitude_matches_oracle(ctx, case):
    nrow, ncol, D, m, p, q, cplx = case
    ket = synth.random_peps(nrow, ncol, D, seed=nrow * 100 + ncol * 10 + D, complex_=cplx)
    dev = dev_lattice(ket)
    for t in range(3):
        bits = _bits(nrow * ncol, t)
        la_ref, ph_ref = amp.amplitude(ket, bits, m, p, q, seed=7)
        la, ph = hp.peps_amplitude(ctx, dev, bits, rank=m, oversample=p, power_iters=q, seed=7)
        assert abs(la - la_ref) <= 1e-10 * max(1.0, abs(la_ref))
        assert abs(ph - ph_ref) <= 1e-10


@pytest.mark.parametrize("case", [CASES[1], CASES[4], CASES[5], CASES[7]],
                         ids=lambda c: "x".join(map(str, c[:3])) + ("c" if c[6] else ""))
def test_batched_amplitudes_match_oracle(ctx, case):
    """A batch of basis states in lockstep, including a state with an exactly zero
    slice: every state equals the oracle's single amplitude."""
    nrow, ncol, D, m, p, q, cplx = case
    ket = synth.random_peps(nrow, ncol, D, seed=nrow * 100 + ncol * 10 + D, complex_=cplx)
    ket[0][0] = ket[0][0].copy()
    ket[0][0][..., 1] = 0.0           # states with bit 1 at site (0, 0) have amplitude 0
    states = [_bits(nrow * ncol, t) for t in range(7)]
    states[3][0] = 1
    for st in states[:3] + states[4:]:
        st[0] = 0
    la, ph = hp.peps_amplitudes(ctx, dev_lattice(ket), states, rank=m, oversample=p, power_iters=q, seed=7)
    for t, st in enumerate(states):
        la_ref, ph_ref = amp.amplitude(ket, st, m, p, q, seed=7)
        if t == 3:
            assert la[t] == -np.inf and ph[t] == 0 and la_ref == -np.inf
            continue
        assert abs(la[t] - la_ref) <= 1e-10 * max(1.0, abs(la_ref))
        assert abs(ph[t] - ph_ref) <= 1e-10


def test_exact_regime_equals_state_vector(ctx):
    ket = synth.random_peps(4, 4, 2, seed=21, complex_=True)
    psi = sv.peps_to_statevector(ket)
    dev = dev_lattice(ket)
    for t in range(4):
        bits = _bits(16, 10 + t)
        la, ph = hp.peps_amplitude(ctx, dev, bits, rank=64, oversample=0, power_iters=0)
        assert abs(ph * np.exp(la) - psi[tuple(bits)]) <= 1e-12 * np.abs(psi).max()


def test_zero_slice_and_errors(ctx):
    ket = synth.random_peps(3, 3, 2, seed=4)
    ket[2][0] = ket[2][0].copy()
    ket[2][0][..., 0] = 0.0
    dev = dev_lattice(ket)
    la, ph = hp.peps_amplitude(ctx, dev, [1] * 6 + [0, 1, 1], rank=3, oversample=1, power_iters=1)
    assert la == -np.inf and ph == 0
    la, ph = hp.peps_amplitude(ctx, dev, [1] * 9, rank=3, oversample=1, power_iters=1)
    la_ref, ph_ref = amp.amplitude(ket, [1] * 9, 3, 1, 1, seed=0)
    assert abs(la - la_ref) <= 1e-10 and abs(ph - ph_ref) <= 1e-10
    with pytest.raises(hp.HpepsError):
        hp.peps_amplitude(ctx, dev, [0] * 8 + [2], rank=3)
    with pytest.raises(hp.HpepsError):
        hp.peps_amplitude(ctx, dev, [0] * 8 + [-1], rank=3)


def test_bench_workload_sample(ctx):
    """The timed workload (16 x 16, D = 8, m = 56, p = 8, q = 1: 210 einsumsvds of
    up to 448 x 3584, nonnegative sites), a batch of 4 of its basis states, against
    the oracle.  With random-sign sites this size is ill-conditioned (in the oracle
    alone a 1e-14 relative perturbation of the sites moves log|a| by about 1.5),
    so no rounding-level comparison exists there; nonnegative sites have no
    cancellation, and at k = 64 every sketch panel keeps full numerical rank
    (smallest singular value above 1e-12 of the largest)."""
    ket = [[np.abs(t) for t in row] for row in synth.random_peps(16, 16, 8, seed=0)]
    states = [_bits(256, t) for t in range(4)]
    la, ph = hp.peps_amplitudes(ctx, dev_lattice(ket), states, rank=56, oversample=8, power_iters=1, seed=0)
    for t in (0, 3):
        la_ref, ph_ref = amp.amplitude(ket, states[t], 56, 8, 1, seed=0)
        assert abs(la[t] - la_ref) <= 1e-10 * max(1.0, abs(la_ref))
        assert abs(ph[t] - ph_ref) <= 1e-10


def test_rank_deficient_sketches(ctx):
    """Sketch panels of numerically lower rank than k (nonnegative 8 x 8, D = 4 sites at
    k = 72: 7 of 42 panels with condition number beyond 1e15).  A Gram-based factorization
    cannot resolve their weak and null directions (with the shifted CholeskyQR passes alone
    the amplitude differed from the oracle by about 4e-9 relative); the first Cholesky pass
    flags them and the Householder fallback orthogonalizes them, as the oracle's QR does,
    so the amplitude matches at the FP64 tolerance."""
    ket = [[np.abs(t) for t in row] for row in synth.random_peps(8, 8, 4, seed=0)]
    bits = _bits(64, 0)
    la_ref, ph_ref = amp.amplitude(ket, bits, 64, 8, 1, seed=0)
    hp.get_info(ctx)
    la, ph = hp.peps_amplitude(ctx, dev_lattice(ket), bits, rank=64, oversample=8, power_iters=1, seed=0)
    assert hp.get_info(ctx)["orth_householder"] >= 1
    assert abs(la - la_ref) <= 1e-10 * max(1.0, abs(la_ref))
    assert abs(ph - ph_ref) <= 1e-10
