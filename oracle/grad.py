"""Gradient reference for einsumsvd (test infrastructure only).

A plain torch-CPU (float64 / complex128) restatement of the randomized SVD of
Alg. 4 on the pair network (as a chain of contractions) and on the explicit
matrix of any network given by subscripts (Sec. II-C), differentiated by torch
autograd with the sketch held fixed: every QR (Householder, torch.linalg.qr) and the final SVD
(torch.linalg.svd) are differentiated as they stand.  Nothing here is shared
with the GPU path; the inputs come from ``synth`` and the sketch from
``oracle.sketch``.

With ``pair_einsumsvd_vjp`` the loss is a linear form of the outputs
themselves (U, sigma, and R = V^* or diag(s) V^*), so it depends on the
canonical phase of the singular pairs and exercises its derivative.

Gradients follow torch's convention for complex inputs (the conjugate
Wirtinger derivative, dL/dRe + i dL/dIm of a real loss).
"""
import numpy as np
import torch

from .rsvd import gauge_vector


def pair_apply(Bl, Br, T1, T2):
    """A X and A^* Y for the pair network A[(a,x,X),(y,Y,c)] (see oracle.network), as
    pairwise contractions of torch tensors, with the dim-1 outer legs dropped."""
    t1, t1b = T1[:, :, 0, :, :], T1[:, :, 0, :, :].conj()
    t2, t2b = T2[:, :, :, 0, :], T2[:, :, :, 0, :].conj()
    a, u, U, b = Bl.shape
    _, v, V, c = Br.shape
    x, y = t1.shape[1], t2.shape[1]
    rows, cols = a * x * x, y * y * c

    def fwd(Om):
        k = Om.shape[1]
        W = torch.einsum("vyhq,yYcj->vhqYcj", t2, Om.reshape(y, y, c, k))
        W = torch.einsum("VYHq,vhqYcj->vhVHcj", t2b, W)
        W = torch.einsum("bvVc,vhVHcj->bhHj", Br, W)
        W = torch.einsum("auUb,bhHj->auUhHj", Bl, W)
        W = torch.einsum("uxhp,auUhHj->axpUHj", t1, W)
        return torch.einsum("UXHp,axpUHj->axXj", t1b, W).reshape(rows, k)

    def adj(P):
        k = P.shape[1]
        W = torch.einsum("UXHp,axXj->axpUHj", t1b.conj(), P.reshape(a, x, x, k))
        W = torch.einsum("uxhp,axpUHj->auUhHj", t1.conj(), W)
        W = torch.einsum("auUb,auUhHj->bhHj", Bl.conj(), W)
        W = torch.einsum("bvVc,bhHj->vhVHcj", Br.conj(), W)
        W = torch.einsum("VYHq,vhVHcj->vhqYcj", t2b.conj(), W)
        return torch.einsum("vyhq,vhqYcj->yYcj", t2.conj(), W).reshape(cols, k)

    return fwd, adj, rows, cols


def fix_gauge(U, s, Vh):
    """The canonical phase of each singular pair (as oracle.rsvd.fix_gauge): the
    projection of U[:, i] on the fixed vector w is made real positive and V^*[i]
    counter-rotated.  Differentiated like every other step, so losses that do
    depend on the phase get its derivative."""
    w = torch.tensor(gauge_vector(U.shape[0]), dtype=U.dtype)
    z = w @ U
    ph = z / z.abs()
    return U * ph.conj()[None, :], s, ph[:, None] * Vh


def randomized_svd(fwd, adj, m, q, omega):
    """Alg. 4 with a fixed sketch: returns U, s, Vh (m' = min(m, k) triplets) in
    the canonical phase."""
    P = torch.linalg.qr(fwd(omega))[0]
    for _ in range(q):
        Q = torch.linalg.qr(adj(P))[0]
        P = torch.linalg.qr(fwd(Q))[0]
    B = adj(P).conj().T                       # P^* A
    Ut, s, Vh = torch.linalg.svd(B, full_matrices=False)
    mp = min(m, omega.shape[1])
    return fix_gauge(P @ Ut[:, :mp], s[:mp], Vh[:mp])


def pair_einsumsvd_grad(Bl, Br, T1, T2, m, q, omega, gM, gs):
    """Gradients of the gauge-invariant loss

        L = Re <gM, U diag(s) V^*> + <gs, s>

    with respect to the four input tensors (numpy arrays in, numpy arrays out), and L."""
    dt = torch.complex128 if np.iscomplexobj(Bl) or np.iscomplexobj(T1) else torch.float64
    ts = [torch.tensor(np.asarray(t), dtype=dt, requires_grad=True) for t in (Bl, Br, T1, T2)]
    fwd, adj, _, _ = pair_apply(*ts)
    U, s, Vh = randomized_svd(fwd, adj, m, q, torch.tensor(omega, dtype=dt))
    M = (U * s.to(dt)) @ Vh
    L = torch.real((torch.tensor(gM, dtype=dt).conj() * M).sum()) + (torch.tensor(gs) * s).sum()
    L.backward()
    return [t.grad.numpy() for t in ts], float(L.detach())


def pair_einsumsvd_loss(Bl, Br, T1, T2, m, q, omega, gM, gs):
    """The loss of pair_einsumsvd_grad alone (for finite differences)."""
    dt = torch.complex128 if np.iscomplexobj(Bl) or np.iscomplexobj(T1) else torch.float64
    with torch.no_grad():
        ts = [torch.tensor(np.asarray(t), dtype=dt) for t in (Bl, Br, T1, T2)]
        fwd, adj, _, _ = pair_apply(*ts)
        U, s, Vh = randomized_svd(fwd, adj, m, q, torch.tensor(omega, dtype=dt))
        M = (U * s.to(dt)) @ Vh
        return float(torch.real((torch.tensor(gM, dtype=dt).conj() * M).sum())
                     + (torch.tensor(gs) * s).sum())


def pair_einsumsvd_vjp(Bl, Br, T1, T2, m, q, omega, right, dU, ds, dR):
    """Gradients of L = Re<dU, U> + <ds, s> + Re<dR, R> with R = V^* (right False) or
    diag(s) V^* (right True), U: rows x m', R: m' x cols; returns the four gradients."""
    dt = torch.complex128 if np.iscomplexobj(Bl) or np.iscomplexobj(T1) else torch.float64
    ts = [torch.tensor(np.asarray(t), dtype=dt, requires_grad=True) for t in (Bl, Br, T1, T2)]
    fwd, adj, _, _ = pair_apply(*ts)
    U, s, Vh = randomized_svd(fwd, adj, m, q, torch.tensor(omega, dtype=dt))
    R = s.to(dt)[:, None] * Vh if right else Vh
    L = (torch.real((torch.tensor(dU, dtype=dt).conj() * U).sum())
         + (torch.tensor(ds) * s).sum()
         + torch.real((torch.tensor(dR, dtype=dt).conj() * R).sum()))
    L.backward()
    return [t.grad.numpy() for t in ts]


def network_apply(subscripts, ts, conj):
    """A X and A^* Y for the network `subscripts` ("ab,bc->a|c") over the torch tensors ts
    (operand i conjugated where conj[i]): the matrix A[(row legs), (column legs)] of the
    network (Sec. II-C) contracted explicitly."""
    lhs, rhs = subscripts.split("->")
    left, right = rhs.split("|")
    ops = [t.conj() if c else t for t, c in zip(ts, conj)]
    A = torch.einsum(lhs + "->" + left + right, *ops)
    rows = int(np.prod(A.shape[:len(left)]))
    cols = int(np.prod(A.shape[len(left):]))
    A = A.reshape(rows, cols)
    return (lambda X: A @ X), (lambda Y: A.conj().T @ Y), rows, cols


def network_einsumsvd_vjp(subscripts, tensors, conj, m, q, omega, right, dU, ds, dR):
    """Gradients of L = Re<dU, U> + <ds, s> + Re<dR, R> (R = V^* or diag(s) V^*, U: rows x m',
    R: m' x cols) of Alg. 4 with the fixed sketch omega on the network's matrix, with respect
    to every operand (numpy arrays in and out; conjugate-Wirtinger for complex operands)."""
    cplx = any(np.iscomplexobj(t) for t in tensors) or np.iscomplexobj(omega)
    dt = torch.complex128 if cplx else torch.float64
    ts = [torch.tensor(np.asarray(t), dtype=dt, requires_grad=True) for t in tensors]
    fwd, adj, _, _ = network_apply(subscripts, ts, conj or [False] * len(ts))
    U, s, Vh = randomized_svd(fwd, adj, m, q, torch.tensor(omega, dtype=dt))
    R = s.to(dt)[:, None] * Vh if right else Vh
    L = (torch.real((torch.tensor(dU, dtype=dt).conj() * U).sum())
         + (torch.tensor(ds) * s).sum()
         + torch.real((torch.tensor(dR, dtype=dt).conj() * R).sum()))
    L.backward()
    return [t.grad.numpy() for t in ts]


def network_einsumsvd_vjp_loss(subscripts, tensors, conj, m, q, omega, right, dU, ds, dR):
    """The loss of network_einsumsvd_vjp alone (for finite differences)."""
    cplx = any(np.iscomplexobj(t) for t in tensors) or np.iscomplexobj(omega)
    dt = torch.complex128 if cplx else torch.float64
    with torch.no_grad():
        ts = [torch.tensor(np.asarray(t), dtype=dt) for t in tensors]
        fwd, adj, _, _ = network_apply(subscripts, ts, conj or [False] * len(ts))
        U, s, Vh = randomized_svd(fwd, adj, m, q, torch.tensor(omega, dtype=dt))
        R = s.to(dt)[:, None] * Vh if right else Vh
        return float(torch.real((torch.tensor(dU, dtype=dt).conj() * U).sum())
                     + (torch.tensor(ds) * s).sum()
                     + torch.real((torch.tensor(dR, dtype=dt).conj() * R).sum()))
