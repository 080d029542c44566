"""GPU parity of the einsumsvd adjoint (reverse sweep of Alg. 4 on the pair
network, hpeps_einsumsvd_pair_backward) against the torch-CPU autograd oracle
on the same seeded inputs and the same sketch.

The loss is L = Re<gM, U diag(s) V^*> + <gs, s> with seeded cotangents; the GPU
side gets the cotangents of its own outputs (U, sigma, R) by the chain rule
written out below for each absorb mode.  Tolerance: max abs error within
1e-9 of the largest gradient entry (FP64 / complex128)."""
import numpy as np
import pytest

import synth
from oracle import grad as og
from oracle.network import pair_operator
from oracle.sketch import sketch as oracle_sketch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _instances(m, D, d, B, cplx, seed):
    inst = [synth.pair_instance(m, D, d, seed=seed, instance=i, complex_=cplx) for i in range(B)]
    return inst, [np.stack([t[j] for t in inst]) for j in range(4)]


def _output_cotangents(U, s, R, gM, gs, absorb):
    """Cotangents of (U, sigma, R) for L = Re<gM, U diag(s) V^*> + <gs, s>:
    RIGHT: M = U R; NONE: M = U diag(s) R (R = V^*)."""
    if absorb == hp.ABSORB_RIGHT:
        return gM @ R.conj().T, gs, U.conj().T @ gM
    dU = gM @ (s[:, None] * R).conj().T
    dR = s[:, None] * (U.conj().T @ gM)
    ds = gs + np.real(np.einsum("ri,rc,ic->i", U.conj(), gM, R.conj()))
    return dU, ds, dR


CASES = [  # m, D, d, rank, p, q, complex, absorb
    (4, 2, 2, 6, 3, 0, False, "none"),
    (4, 2, 2, 6, 3, 2, False, "right"),
    (6, 3, 2, 10, 6, 1, False, "none"),
    (6, 3, 2, 10, 6, 1, True, "right"),
    (5, 3, 3, 12, 4, 2, True, "none"),
    (9, 4, 2, 20, 8, 1, False, "right"),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "m%d_D%d_d%d_r%d_p%d_q%d_%s_%s" % (
    c[0], c[1], c[2], c[3], c[4], c[5], "c" if c[6] else "r", c[7]))
def test_pair_backward_parity(ctx, case):
    m, D, d, rank, p, q, cplx, ab = case
    absorb = hp.ABSORB_RIGHT if ab == "right" else hp.ABSORB_NONE
    B = 2
    inst, st = _instances(m, D, d, B, cplx, seed=31)
    op0 = pair_operator(*inst[0])
    rows, cols = op0.n_rows, op0.n_cols
    k = min(rank + p, rows, cols)
    mp = min(rank, k)
    dev = [_dev(t) for t in st]
    U, s, R = hp.einsumsvd_pair(ctx, *dev, rank=rank, oversample=p, power_iters=q, seed=2,
                                stream_id=40, absorb=absorb)
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    rng = np.random.default_rng(17)
    dUs, dss, dRs, refs = [], [], [], []
    for i in range(B):
        gM = rng.standard_normal((rows, cols))
        if cplx:
            gM = gM + 1j * rng.standard_normal((rows, cols))
        gs = rng.standard_normal(mp)
        dU, ds, dR = _output_cotangents(U[i].reshape(rows, mp), s[i], R[i].reshape(mp, cols),
                                        gM, gs, absorb)
        dUs.append(dU.reshape(m, D, D, mp))
        dss.append(ds)
        dRs.append(dR.reshape(mp, D, D, m))
        om = oracle_sketch(2, 40 + i, cols, k)
        refs.append(og.pair_einsumsvd_grad(*inst[i], rank, q, om, gM, gs)[0])
    g = hp.einsumsvd_pair_backward(ctx, *dev, _dev(np.stack(dUs)), _dev(np.stack(dss)),
                                   _dev(np.stack(dRs)), rank=rank, oversample=p, power_iters=q,
                                   seed=2, stream_id=40, absorb=absorb)
    g = [t.cpu().numpy() for t in g]
    for i in range(B):
        for j in range(4):
            ref = refs[i][j]
            err = np.max(np.abs(g[j][i] - ref)) / np.max(np.abs(ref))
            assert err < 1e-9, (i, j, err)


def test_pair_backward_autograd(ctx):
    """The torch.autograd binding: loss built from the GPU outputs with torch ops,
    gradients from loss.backward() equal the oracle's."""
    m, D, d, rank, p, q = 5, 3, 2, 8, 4, 1
    inst, st = _instances(m, D, d, 1, False, seed=44)
    op0 = pair_operator(*inst[0])
    rows, cols = op0.n_rows, op0.n_cols
    k = min(rank + p, rows, cols)
    xs = [_dev(t).requires_grad_(True) for t in st]
    U, s, R = hp.einsumsvd_pair_autograd(ctx, *xs, rank=rank, oversample=p, power_iters=q,
                                         seed=6, stream_id=1, absorb=hp.ABSORB_RIGHT)
    rng = np.random.default_rng(3)
    gM = rng.standard_normal((rows, cols))
    gs = rng.standard_normal(rank)
    M = U.reshape(rows, rank) @ R.reshape(rank, cols)
    loss = (_dev(gM) * M).sum() + (_dev(gs) * s[0]).sum()
    loss.backward()
    om = oracle_sketch(6, 1, cols, k)
    ref, _ = og.pair_einsumsvd_grad(*inst[0], rank, q, om, gM, gs)
    for j in range(4):
        got = xs[j].grad.cpu().numpy()[0]
        assert np.max(np.abs(got - ref[j])) < 1e-9 * np.max(np.abs(ref[j]))


def test_pair_backward_rejects_carry(ctx):
    inst, st = _instances(4, 2, 2, 1, False, seed=1)
    dev = [_dev(t) for t in st]
    dU = torch.zeros((1, 4, 2, 2, 4), dtype=torch.float64, device="cuda")
    dR = torch.zeros((1, 4, 2, 2, 4), dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HpepsError):
        hp.einsumsvd_pair_backward(ctx, *dev, dU, None, dR, rank=4, absorb=hp.ABSORB_CARRY)


@pytest.mark.parametrize("cplx,ab", [(True, "none"), (True, "right"), (False, "right")])
def test_pair_backward_phase_dependent(ctx, cplx, ab):
    """Cotangents put directly on U, sigma and R: the loss depends on the canonical
    phase of the singular pairs (complex), so the adjoint's phase term is exercised."""
    m, D, d, rank, p, q = 5, 3, 2, 9, 5, 1
    absorb = hp.ABSORB_RIGHT if ab == "right" else hp.ABSORB_NONE
    B = 2
    inst, st = _instances(m, D, d, B, cplx, seed=77)
    op0 = pair_operator(*inst[0])
    rows, cols = op0.n_rows, op0.n_cols
    k = min(rank + p, rows, cols)
    rng = np.random.default_rng(4)

    def draw(*s):
        x = rng.standard_normal(s)
        return x + 1j * rng.standard_normal(s) if cplx else x

    dUs = [draw(rows, rank) for _ in range(B)]
    dss = [rng.standard_normal(rank) for _ in range(B)]
    dRs = [draw(rank, cols) for _ in range(B)]
    dev = [_dev(t) for t in st]
    g = hp.einsumsvd_pair_backward(
        ctx, *dev, _dev(np.stack([x.reshape(m, D, D, rank) for x in dUs])), _dev(np.stack(dss)),
        _dev(np.stack([x.reshape(rank, D, D, m) for x in dRs])), rank=rank, oversample=p,
        power_iters=q, seed=5, stream_id=2, absorb=absorb)
    g = [t.cpu().numpy() for t in g]
    for i in range(B):
        om = oracle_sketch(5, 2 + i, cols, k)
        ref = og.pair_einsumsvd_vjp(*inst[i], rank, q, om, ab == "right", dUs[i], dss[i], dRs[i])
        for j in range(4):
            err = np.max(np.abs(g[j][i] - ref[j])) / np.max(np.abs(ref[j]))
            assert err < 1e-9, (i, j, err)
