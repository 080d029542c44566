"""The allocation-free two-site gate update (hpeps_apply_two_site_gate_noalloc, its
buffers in the library's static device scratch) against the allocating entry point
(hpeps_apply_two_site_gate) through the C ABI: identical sites and singular values on
two calls in a row, the second on a smaller lattice with a smaller bond, and again after
an allocating call in between."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


def _lattice(nrow, ncol, D, seed):
    return [[torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in row]
            for row in synth.random_peps(nrow, ncol, D, seed=seed)]


def _gate(seed):
    Hb = synth.tfi_bond_hamiltonians(2, 2, 1.0, 3.0)[((0, 0), (0, 1))]
    G = synth.bond_gate(Hb, 0.1 + 0.01 * seed)
    return torch.from_numpy(np.ascontiguousarray(np.real(G))).cuda()


def _same(ctx, nrow, ncol, D, i, j, axis, max_rank, seed):
    sites = _lattice(nrow, ncol, D, seed)
    G = _gate(seed)
    ref, sref = hp.apply_two_site_gate(ctx, sites, i, j, axis, G, max_rank)
    got, sgot = hp.apply_two_site_gate(ctx, sites, i, j, axis, G, max_rank, noalloc=True)
    assert sgot.shape == sref.shape
    s_ref = sref.cpu().numpy()
    assert np.max(np.abs(sgot.cpu().numpy() - s_ref)) <= 1e-12 * s_ref[0]
    for r in range(nrow):
        for c in range(ncol):
            a, b = ref[r][c].cpu().numpy(), got[r][c].cpu().numpy()
            assert a.shape == b.shape
            assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.max(np.abs(a)))
    return s_ref


def test_noalloc_gate_matches_allocating_call():
    ctx = hp.Context(0)
    _same(ctx, 3, 3, 4, 1, 1, 0, 4, seed=0)           # horizontal bulk bond, D = 4
    _same(ctx, 2, 2, 2, 0, 0, 1, 2, seed=1)           # smaller: vertical edge bond, D = 2
    _same(ctx, 3, 4, 3, 1, 2, 1, 3, seed=2)           # after both, a third shape


def test_noalloc_gate_rejects_bad_arguments():
    ctx = hp.Context(0)
    sites = _lattice(2, 2, 2, 3)
    with pytest.raises(hp.HpepsError):
        hp.apply_two_site_gate(ctx, sites, 0, 1, 0, _gate(0), 2, noalloc=True)   # bond outside
    with pytest.raises(hp.HpepsError):
        hp.apply_two_site_gate(ctx, sites, 0, 0, 0, _gate(0), 64, noalloc=True)  # max_rank too large
