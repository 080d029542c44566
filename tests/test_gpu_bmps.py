"""GPU parity of boundary-MPS contraction (Algs. 2-3): peps_norm and
boundary_contract_row against the oracle on the same seeded lattices and
sketches.  Norms are compared in log space: |log N_gpu - log N_oracle| <= 1e-10
(FP64 / complex128 sketches), <= 1e-4 for FP32 sketches."""
import numpy as np
import pytest

import synth
from oracle import bmps, statevector as sv
from oracle.sketch import stream_id

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def dev_lattice(peps):
    return [[torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in row] for row in peps]


def test_c1_exact_regime_equals_brute_force(ctx):
    peps = synth.random_peps(4, 4, D=2, seed=0)
    psi = sv.peps_to_statevector(peps)
    ref = np.log(np.vdot(psi, psi).real)
    ln, ph = hp.peps_norm(ctx, dev_lattice(peps), rank=64, oversample=8, power_iters=1)
    assert abs(ln - ref) < 1e-10 and abs(ph - 1) < 1e-12


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_c1_truncated_parity(ctx, seed):
    """The 4x4 norm with m=4, p=4, q=1: GPU equals the oracle's randomized
    contraction; the error against the brute-force norm is only reported."""
    peps = synth.random_peps(4, 4, D=2, seed=seed)
    lo, po = bmps.peps_norm(peps, m=4, p=4, q=1, seed=seed)
    ln, ph = hp.peps_norm(ctx, dev_lattice(peps), rank=4, oversample=4, power_iters=1, seed=seed)
    assert abs(ln - lo) < 1e-10 and abs(ph - po) < 1e-10


CASES = [
    # nrow, ncol, D, m, p, q, complex
    (3, 3, 2, 3, 2, 1, False),
    (3, 4, 2, 5, 3, 0, True),
    (4, 3, 3, 6, 4, 2, False),
    (5, 4, 2, 6, 2, 1, True),
    (2, 5, 3, 4, 4, 1, False),
    (1, 4, 2, 4, 4, 1, True),
    (6, 6, 2, 8, 4, 1, False),
]


@pytest.mark.parametrize("case", CASES)
def test_norm_parity(ctx, case):
    nrow, ncol, D, m, p, q, cplx = case
    peps = synth.random_peps(nrow, ncol, D=D, seed=nrow * 10 + ncol, complex_=cplx)
    lo, po = bmps.peps_norm(peps, m=m, p=p, q=q, seed=7)
    ln, ph = hp.peps_norm(ctx, dev_lattice(peps), rank=m, oversample=p, power_iters=q, seed=7)
    assert abs(ln - lo) < 1e-10
    assert abs(ph - po) < 1e-10


def test_norm_of_two_different_states(ctx):
    ket = synth.random_peps(3, 4, D=2, seed=1, complex_=True)
    bra = synth.random_peps(3, 4, D=2, seed=2, complex_=True)
    lo, po = bmps.peps_norm(ket, m=4, p=2, q=1, seed=3, bra=bra)
    ln, ph = hp.peps_norm(ctx, dev_lattice(ket), dev_lattice(bra), rank=4, oversample=2,
                          power_iters=1, seed=3)
    assert abs(ln - lo) < 1e-10 and abs(ph - po) < 1e-10


def test_norm_fp32_sketch(ctx):
    peps = synth.random_peps(5, 5, D=2, seed=11)
    lo, _ = bmps.peps_norm(peps, m=6, p=4, q=2, seed=0)
    ln, _ = hp.peps_norm(ctx, dev_lattice(peps), rank=6, oversample=4, power_iters=2, seed=0,
                         precision="f32")
    assert abs(ln - lo) < 1e-4


@pytest.mark.parametrize("m,p,q", [(6, 4, 2), (16, 8, 2)])
def test_norm_bf16_sketch(ctx, m, p, q):
    """BF16 operator applications: the log norm within 3e-2 of the FP64 oracle."""
    peps = synth.random_peps(5, 5, D=2, seed=11)
    lo, _ = bmps.peps_norm(peps, m=m, p=p, q=q, seed=0)
    ln, _ = hp.peps_norm(ctx, dev_lattice(peps), rank=m, oversample=p, power_iters=q, seed=0,
                         precision="bf16")
    assert abs(ln - lo) < 3e-2


def test_norm_tiny_scale_is_finite(ctx):
    peps = synth.random_peps(4, 4, D=2, seed=4)
    ref, _ = hp.peps_norm(ctx, dev_lattice(peps), rank=4, oversample=4, power_iters=1)
    tiny = [[t * 1e-200 for t in row] for row in peps]
    ln, _ = hp.peps_norm(ctx, dev_lattice(tiny), rank=4, oversample=4, power_iters=1)
    assert np.isfinite(ln) and abs(ln - (ref + 32 * np.log(1e-200))) < 1e-8


def _mps_full(tensors, log_scale):
    """Contract a boundary MPS [mL,x,X,mR] over its bonds (gauge invariant)."""
    v = np.ones((1, 1))
    for S in tensors:
        v = np.einsum("pa,axXb->pxXb", v, S).reshape(-1, S.shape[3])
    return v.reshape(-1) * np.exp(log_scale)


@pytest.mark.parametrize("direction", [0, 1])
@pytest.mark.parametrize("cplx", [False, True])
def test_boundary_contract_row(ctx, direction, cplx):
    nrow, ncol, D, m, p, q = 3, 4, 2, 3, 2, 1
    peps = synth.random_peps(nrow, ncol, D=D, seed=5, complex_=cplx)
    bnd, ls0 = bmps.first_row_boundary(peps[0], peps[0])
    sids = [stream_id(0, nrow, ncol, 1, j) for j in range(ncol)]
    ref, ls, _ = bmps.absorb_row(bnd, peps[1], peps[1], direction, m, p, q, 9, sids)
    dbnd = [torch.from_numpy(np.ascontiguousarray(S)).cuda() for S in bnd]
    out, lsg = hp.boundary_contract_row(ctx, dbnd, dev_lattice(peps), row=1,
                                        direction=direction, rank=m, oversample=p, power_iters=q,
                                        seed=9, stream_id=sids[0])
    got = [t.cpu().numpy() for t in out]
    for a, b in zip(got, ref):
        assert a.shape == b.shape
    fa, fb = _mps_full(got, lsg), _mps_full(ref, ls)
    assert np.max(np.abs(fa - fb)) < 1e-10 * np.max(np.abs(fb))
