"""Pins of the gradient oracle (oracle/grad.py) against what does not depend on
autograd: central finite differences of the loss, and the closed form of the
exact-SVD case (sketch width = operator size, where U diag(s) V^* = A and the
derivative of sigma_1 is Re(u_1 v_1^*)).
"""
import numpy as np
import pytest

import synth
from oracle import grad as og
from oracle.network import pair_operator
from oracle.sketch import sketch as oracle_sketch

torch = pytest.importorskip("torch")


def _cotangents(rng, rows, cols, mp, cplx):
    gM = rng.standard_normal((rows, cols))
    if cplx:
        gM = gM + 1j * rng.standard_normal((rows, cols))
    return gM, rng.standard_normal(mp)


def _fd_check(inst, m, q, omega, gM, gs, n_probe=12, h=1e-6, seed=0):
    grads, _ = og.pair_einsumsvd_grad(*inst, m, q, omega, gM, gs)
    rng = np.random.default_rng(seed)
    worst = 0.0
    for ti, t in enumerate(inst):
        scale = np.max(np.abs(grads[ti]))
        for _ in range(n_probe):
            idx = tuple(rng.integers(0, s) for s in t.shape)
            parts = [1.0] + ([1j] if np.iscomplexobj(t) else [])
            fd = 0.0
            for part in parts:
                def loss_at(delta):
                    ts = [x.copy() for x in inst]
                    ts[ti][idx] += delta * part
                    return og.pair_einsumsvd_loss(*ts, m, q, omega, gM, gs)
                d = (loss_at(h) - loss_at(-h)) / (2 * h)
                fd = fd + d * part      # dL/dRe + i dL/dIm
            worst = max(worst, abs(fd - grads[ti][idx]) / scale)
    return worst


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("q", [0, 2])
def test_grad_oracle_finite_differences(cplx, q):
    """Truncated case (m' < k < n): every QR and the SVD enter the derivative."""
    m, D, d, rank, p = 3, 2, 2, 4, 3
    inst = synth.pair_instance(m, D, d, seed=21, instance=q, complex_=cplx)
    op = pair_operator(*inst)
    k = min(rank + p, op.n_rows, op.n_cols)
    omega = oracle_sketch(4, 9, op.n_cols, k)
    gM, gs = _cotangents(np.random.default_rng(5), op.n_rows, op.n_cols, rank, cplx)
    assert _fd_check(inst, rank, q, omega, gM, gs) < 1e-6


def test_grad_oracle_exact_svd_closed_form():
    """k = n: U diag(s) V^* = A exactly, so the gradient of Re<gM, A> + s_1 is the
    gradient of the linear map A(tensors) against gM + Re(u_1 v_1^*), computed here
    from the explicit operator without any factorization in the derivative."""
    m, D, d = 2, 2, 2
    inst = synth.pair_instance(m, D, d, seed=3, instance=1)
    op = pair_operator(*inst)
    n = op.n_rows
    omega = oracle_sketch(1, 2, op.n_cols, n)
    gM = np.random.default_rng(8).standard_normal((n, op.n_cols))
    gs = np.zeros(n)
    gs[0] = 1.0
    grads, _ = og.pair_einsumsvd_grad(*inst, n, 1, omega, gM, gs)
    A = op.explicit()
    u, s, vh = np.linalg.svd(A)
    W = gM + np.outer(u[:, 0], vh[0])          # dL/dA for a real operator
    # dL/dtensor = sum_rc W[r,c] dA[r,c]/dtensor; A is multilinear in the six slots
    # (a site tensor fills its ket and its bra slot), so the derivative along the basis
    # direction e_idx is the sum over the tensor's slots of A with that slot set to e_idx
    Bl, Br, T1, T2 = inst
    assert np.allclose(_explicit(Bl, Br, T1, T1, T2, T2), A, atol=1e-14)
    rng = np.random.default_rng(0)
    for ti, t in enumerate(inst):
        for _ in range(10):
            idx = tuple(rng.integers(0, s_) for s_ in t.shape)
            e = np.zeros_like(t)
            e[idx] = 1.0
            if ti == 0:
                dA = _explicit(e, Br, T1, T1, T2, T2)
            elif ti == 1:
                dA = _explicit(Bl, e, T1, T1, T2, T2)
            elif ti == 2:
                dA = _explicit(Bl, Br, e, T1, T2, T2) + _explicit(Bl, Br, T1, e, T2, T2)
            else:
                dA = _explicit(Bl, Br, T1, T1, e, T2) + _explicit(Bl, Br, T1, T1, T2, e)
            ref = np.sum(W * dA)
            assert abs(ref - grads[ti][idx]) < 1e-9 * np.max(np.abs(grads[ti]))


def _explicit(Bl, Br, t1k, t1b, t2k, t2b):
    """A[(a,x,X),(y,Y,c)] = sum Bl[a,u,U,b] Br[b,v,V,c] T1[u,x,h,p] T1b[U,X,H,p]
    T2[v,y,h,q] T2b[V,Y,H,q] (dim-1 outer legs dropped), real tensors."""
    a1, b1 = t1k[:, :, 0], t1b[:, :, 0]
    a2, b2 = t2k[:, :, :, 0], t2b[:, :, :, 0]
    A = np.einsum("auUb,bvVc,uxhp,UXHp,vyhq,VYHq->axXyYc", Bl, Br, a1, b1, a2, b2)
    m, D = Bl.shape[0], Bl.shape[1]
    return A.reshape(m * D * D, -1)


def _vjp_loss(inst, m, q, omega, right, dU, ds, dR):
    dt = torch.complex128 if np.iscomplexobj(inst[0]) else torch.float64
    with torch.no_grad():
        fwd, adj, _, _ = og.pair_apply(*[torch.tensor(t, dtype=dt) for t in inst])
        U, s, Vh = og.randomized_svd(fwd, adj, m, q, torch.tensor(omega, dtype=dt))
        R = s.to(dt)[:, None] * Vh if right else Vh
        return float(torch.real((torch.tensor(dU, dtype=dt).conj() * U).sum())
                     + (torch.tensor(ds) * s).sum()
                     + torch.real((torch.tensor(dR, dtype=dt).conj() * R).sum()))


@pytest.mark.parametrize("right", [False, True])
def test_grad_oracle_phase_dependent_loss(right):
    """A loss linear in U and R themselves depends on the canonical phase of the
    singular pairs (complex case): the oracle's gradient, which differentiates the
    phase choice, must match central finite differences of the loss."""
    m, D, d, rank, p, q = 3, 2, 2, 4, 3, 1
    inst = synth.pair_instance(m, D, d, seed=13, instance=0, complex_=True)
    op = pair_operator(*inst)
    k = min(rank + p, op.n_rows, op.n_cols)
    omega = oracle_sketch(7, 3, op.n_cols, k)
    rng = np.random.default_rng(2)
    c = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    dU, ds, dR = c(op.n_rows, rank), rng.standard_normal(rank), c(rank, op.n_cols)
    grads = og.pair_einsumsvd_vjp(*inst, rank, q, omega, right, dU, ds, dR)
    rng2 = np.random.default_rng(1)
    h = 1e-6
    for ti, t in enumerate(inst):
        scale = np.max(np.abs(grads[ti]))
        for _ in range(8):
            idx = tuple(rng2.integers(0, s_) for s_ in t.shape)
            fd = 0.0
            for part in (1.0, 1j):
                vals = []
                for sgn in (1, -1):
                    ts = [x.copy() for x in inst]
                    ts[ti][idx] += sgn * h * part
                    vals.append(_vjp_loss(ts, rank, q, omega, right, dU, ds, dR))
                fd = fd + (vals[0] - vals[1]) / (2 * h) * part
            assert abs(fd - grads[ti][idx]) < 1e-6 * scale, (ti, idx)


PAIR_NET = "auUb,bvVc,uxhp,UXHp,vyhq,VYHq->axX|yYc"


@pytest.mark.parametrize("cplx", [False, True])
@pytest.mark.parametrize("right", [False, True])
def test_network_grad_oracle_equals_pair_oracle(cplx, right):
    """The network gradient oracle (explicit matrix of any network) on the pair network
    equals the pair oracle (the operator as a chain of contractions): T1 and T2 enter twice,
    as ket and as conjugated bra, and their gradients are the sums of the two entries'."""
    m, D, d, rank, p, q = 3, 2, 2, 4, 3, 1
    inst = synth.pair_instance(m, D, d, seed=17, instance=0, complex_=cplx)
    Bl, Br, T1, T2 = inst
    op = pair_operator(*inst)
    k = min(rank + p, op.n_rows, op.n_cols)
    omega = oracle_sketch(5, 2, op.n_cols, k)
    rng = np.random.default_rng(4)
    c = (lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)) if cplx else \
        (lambda *s: rng.standard_normal(s))
    dU, ds, dR = c(op.n_rows, rank), rng.standard_normal(rank), c(rank, op.n_cols)
    gp = og.pair_einsumsvd_vjp(*inst, rank, q, omega, right, dU, ds, dR)
    t1, t2 = T1[:, :, 0], T2[:, :, :, 0]
    gn = og.network_einsumsvd_vjp(PAIR_NET, [Bl, Br, t1, t1, t2, t2], [False, False, False, True, False, True],
                                  rank, q, omega, right, dU, ds, dR)
    scale = max(np.max(np.abs(g)) for g in gp)
    assert np.max(np.abs(gn[0] - gp[0])) < 1e-10 * scale
    assert np.max(np.abs(gn[1] - gp[1])) < 1e-10 * scale
    assert np.max(np.abs(gn[2] + gn[3] - gp[2][:, :, 0])) < 1e-10 * scale
    assert np.max(np.abs(gn[4] + gn[5] - gp[3][:, :, :, 0])) < 1e-10 * scale


def test_network_grad_oracle_finite_differences():
    """Central finite differences (Re and Im parts) of the network loss, on a three-operand
    network with a conjugated operand and a truncated sketch (q = 1)."""
    rng = np.random.default_rng(6)
    c = lambda *s: rng.standard_normal(s) + 1j * rng.standard_normal(s)
    A, B, Cc = c(2, 3, 4), c(4, 3, 2), c(2, 5, 2)
    subs, conj = "abc,cde,efa->bd|f", [False, False, True]
    rank, q = 3, 1
    omega = oracle_sketch(3, 1, 5, 4)
    dU, ds, dR = c(9, rank), rng.standard_normal(rank), c(rank, 5)
    inst = [A, B, Cc]
    grads = og.network_einsumsvd_vjp(subs, inst, conj, rank, q, omega, True, dU, ds, dR)
    h = 1e-6
    for ti, t in enumerate(inst):
        scale = np.max(np.abs(grads[ti]))
        for _ in range(6):
            idx = tuple(rng.integers(0, s_) for s_ in t.shape)
            fd = 0.0
            for part in (1.0, 1j):
                vals = []
                for sgn in (1, -1):
                    ts = [x.copy() for x in inst]
                    ts[ti][idx] += sgn * h * part
                    vals.append(og.network_einsumsvd_vjp_loss(subs, ts, conj, rank, q, omega, True, dU, ds, dR))
                fd = fd + (vals[0] - vals[1]) / (2 * h) * part
            assert abs(fd - grads[ti][idx]) < 1e-6 * scale, (ti, idx)
