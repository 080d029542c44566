"""Gradient reference for the boundary-MPS norm and the cached energy
(test infrastructure only).

A torch-CPU (float64 / complex128) restatement of oracle.bmps (Alg. 2, the
zip-up ApproxApply of Alg. 3 with the randomized einsumsvd of Alg. 4) and of
oracle.energy's cached path (Eq. 5 with the environments of Sec. IV-B),
step for step and with the same sketches, so that its forward values equal
the numpy oracle's (like it, the energy runs on the unrescaled sites).
torch autograd then differentiates every step as it stands: the Householder
QRs, the SVD, the canonical phase choice of the singular pairs, and every
Frobenius and sigma_1 rescaling (none of which are constants here).  Nothing
is shared with the GPU path.

Gradients are torch's conjugate Wirtinger gradients (dL/dRe + i dL/dIm) of
the real losses log<psi|psi> and Re E.
"""
import numpy as np
import torch

from .energy import operator_schmidt
from .grad import randomized_svd
from .rsvd import sketch_width
from .sketch import sketch, stream_id

L2R, R2L = 0, 1
TOP, BOTTOM = 0, 1


def _zipup(V, S, T, B):
    """A X and A^* Y of the zip-up operator (oracle.network.zipup_operator)."""
    a, x, X, b, h, H = V.shape
    y, G = T.shape[1], B.shape[3]
    c, g, Y = S.shape[3], T.shape[3], B.shape[1]
    Bc = B.conj()
    rows, cols = (a, x, X), (y, Y, c, g, G)

    def fwd(Om):
        k = Om.shape[1]
        W = torch.einsum("uyhgp,yYcgGj->uhpYcGj", T, Om.reshape(cols + (k,)))
        W = torch.einsum("UYHGp,uhpYcGj->uhUHcj", Bc, W)
        W = torch.einsum("buUc,uhUHcj->bhHj", S, W)
        return torch.einsum("axXbhH,bhHj->axXj", V, W).reshape(a * x * X, k)

    def adj(P):
        k = P.shape[1]
        W = torch.einsum("axXbhH,axXj->bhHj", V.conj(), P.reshape(rows + (k,)))
        W = torch.einsum("buUc,bhHj->uhUHcj", S.conj(), W)
        W = torch.einsum("UYHGp,uhUHcj->uhpYcGj", B, W)
        return torch.einsum("uyhgp,uhpYcGj->yYcgGj", T.conj(), W).reshape(-1, k)

    return fwd, adj, rows, cols


def _mirror_lr_site(T):
    return T.permute(0, 1, 3, 2, 4)


def _mirror_ud_site(T):
    return T.permute(1, 0, 2, 3, 4)


def _mirror_lr_bnd(S):
    return S.permute(3, 1, 2, 0)


def _first_row_boundary(ket_row, bra_row):
    out, log_scale = [], 0.0
    for T, B in zip(ket_row, bra_row):
        S = torch.einsum("udlrp,UDLRp->lLdDrR", T[:1], B[:1].conj())
        l, L, d, Dd, r, R = S.shape
        S = S.reshape(l * L, d, Dd, r * R)
        nrm = torch.linalg.norm(S)
        out.append(S / nrm)
        log_scale = log_scale + torch.log(nrm)
    return out, log_scale


def _zipup_row_l2r(bnd, ket_row, bra_row, m, p, q, seed, sids):
    n = len(ket_row)
    V = torch.einsum("buUc,uyhgp,UYHGp->byYcgG", bnd[0], ket_row[0], bra_row[0].conj())
    nrm = torch.linalg.norm(V)
    V = V / nrm
    log_scale = torch.log(nrm)
    out = []
    for j in range(1, n):
        fwd, adj, rows, cols = _zipup(V, bnd[j], ket_row[j], bra_row[j])
        n_rows, n_cols = int(np.prod(rows)), int(np.prod(cols))
        k = sketch_width(m, p, n_rows, n_cols)
        omega = torch.tensor(sketch(seed, sids[j], n_cols, k), dtype=V.dtype)
        U, s, Vh = randomized_svd(fwd, adj, m, q, omega)
        mp = s.shape[0]
        out.append(U.reshape(rows + (mp,)))
        V = ((s / s[0]).to(V.dtype)[:, None] * Vh).reshape((mp,) + cols)
        log_scale = log_scale + torch.log(s[0])
    a, y, Y, c, g, G = V.shape
    out.append(V.reshape(a, y, Y, c * g * G))
    return out, log_scale


def _absorb_row(bnd, ket_row, bra_row, direction, m, p, q, seed, sids):
    if direction == L2R:
        return _zipup_row_l2r(bnd, ket_row, bra_row, m, p, q, seed, sids)
    out, ls = _zipup_row_l2r([_mirror_lr_bnd(S) for S in reversed(bnd)],
                             [_mirror_lr_site(T) for T in reversed(ket_row)],
                             [_mirror_lr_site(B) for B in reversed(bra_row)],
                             m, p, q, seed, list(reversed(sids)))
    return [_mirror_lr_bnd(S) for S in reversed(out)], ls


def _contract_last_row(bnd, ket_row, bra_row):
    E = torch.ones((1, 1, 1), dtype=bnd[0].dtype)
    log_scale = 0.0
    for S, T, B in zip(bnd, ket_row, bra_row):
        X = torch.einsum("bhH,buUc->hHuUc", E, S)
        X = torch.einsum("hHuUc,uhgp->HUcgp", X, T[:, 0])
        E = torch.einsum("HUcgp,UHGp->cgG", X, B[:, 0].conj())
        nrm = torch.linalg.norm(E)
        E = E / nrm
        log_scale = log_scale + torch.log(nrm)
    return E.reshape(()), log_scale


def _oriented(ket, side):
    if side == TOP:
        return ket
    return [[_mirror_ud_site(T) for T in row] for row in reversed(ket)]


def _boundary_pass(ket, side, m, p, q, seed):
    """Every intermediate boundary MPS of one pass, bra = ket (oracle.bmps.boundary_pass)."""
    nrow, ncol = len(ket), len(ket[0])
    K = _oriented(ket, side)
    bnd, log_scale = _first_row_boundary(K[0], K[0])
    envs, logs = [bnd], [log_scale]
    for t in range(1, nrow - 1):
        orig_row = t if side == TOP else nrow - 1 - t
        direction = L2R if t % 2 == 1 else R2L
        sids = [stream_id(side, nrow, ncol, orig_row, j) for j in range(ncol)]
        bnd, ls = _absorb_row(bnd, K[t], K[t], direction, m, p, q, seed, sids)
        log_scale = log_scale + ls
        envs.append(bnd)
        logs.append(log_scale)
    return envs, logs


def _normalized_sites(layer):
    out, log_scale = [], 0.0
    for row in layer:
        new = []
        for T in row:
            mx = T.abs().max()
            T = T / mx
            nrm = torch.linalg.norm(T)
            new.append(T / nrm)
            log_scale = log_scale + torch.log(nrm) + torch.log(mx)
        out.append(new)
    return out, log_scale


def log_norm(ket, m, p, q, seed):
    """log <psi|psi> by boundary MPS (oracle.bmps.peps_norm with bra = ket), as a
    differentiable torch scalar; ket: rows of torch site tensors."""
    nrow = len(ket)
    kn, lk = _normalized_sites(ket)
    bn, lb = _normalized_sites(ket)
    if nrow == 1:
        bnd, ls = _first_row_boundary(kn[0], bn[0])
        E = torch.ones((1,), dtype=bnd[0].dtype)
        for S in bnd:
            E = E @ S[:, 0, 0, :]
            nrm = torch.linalg.norm(E)
            E, ls = E / nrm, ls + torch.log(nrm)
        return lk + lb + ls + torch.log(E.reshape(()).abs())
    # bra and ket layers are separate rescaled copies of the same tensors
    bnd, log_scale = _first_row_boundary(kn[0], bn[0])
    for t in range(1, nrow - 1):
        direction = L2R if t % 2 == 1 else R2L
        ncol = len(ket[0])
        sids = [stream_id(TOP, nrow, ncol, t, j) for j in range(ncol)]
        bnd, ls = _absorb_row(bnd, kn[t], bn[t], direction, m, p, q, seed, sids)
        log_scale = log_scale + ls
    v, ls = _contract_last_row(bnd, kn[nrow - 1], bn[nrow - 1])
    return lk + lb + log_scale + ls + torch.log(v.abs())


def _col3(L, Tp, T, O, B, Bt):
    TO = torch.einsum("Pp,udlrp->udlrP", O, T)
    X = torch.einsum("tlLb,tuUs->lLbuUs", L, Tp)
    X = torch.einsum("lLbuUs,udlrP->LbUsdrP", X, TO)
    X = torch.einsum("LbUsdrP,UDLRP->bsdrDR", X, B.conj())
    return torch.einsum("bsdrDR,bdDc->srRc", X, Bt)


def _col4(L, Tp, T1, O1, B1, T2, O2, B2, Bt):
    T1O = torch.einsum("Pp,uvlrp->uvlrP", O1, T1)
    T2O = torch.einsum("Qq,vdmnq->vdmnQ", O2, T2)
    X = torch.einsum("tlLmMb,tuUs->lLmMbuUs", L, Tp)
    X = torch.einsum("lLmMbuUs,uvlrP->LmMbUsvrP", X, T1O)
    X = torch.einsum("LmMbUsvrP,UVLRP->mMbsvrVR", X, B1.conj())
    X = torch.einsum("mMbsvrVR,vdmnQ->MbsrVRdnQ", X, T2O)
    X = torch.einsum("MbsrVRdnQ,VDMNQ->bsrRdnDN", X, B2.conj())
    return torch.einsum("bsrRdnDN,bdDc->srRnNc", X, Bt)


def _mirror3(Tp, T, B, Bt):
    return (Tp.permute(3, 1, 2, 0), T.permute(0, 1, 3, 2, 4), B.permute(0, 1, 3, 2, 4),
            Bt.permute(3, 1, 2, 0))


def _norm(x):
    return x / torch.linalg.norm(x)


def _row_terms(top, row, bot, terms_here, d, dt):
    n = len(row)
    I = torch.eye(d, dtype=dt)
    Ls = [torch.ones((1, 1, 1, 1), dtype=dt)]
    for j in range(n):
        Ls.append(_norm(_col3(Ls[-1], top[j], row[j], I, row[j], bot[j])))
    Rs = [torch.ones((1, 1, 1, 1), dtype=dt)]
    for j in reversed(range(n)):
        Tp, T, B, Bt = _mirror3(top[j], row[j], row[j], bot[j])
        Rs.append(_norm(_col3(Rs[-1], Tp, T, I, B, Bt)))
    Rs = Rs[::-1]
    out = []
    for sites, op in terms_here:
        j = sites[0][1]
        if len(sites) == 1:
            O = torch.tensor(op, dtype=dt)
            num = torch.sum(Rs[j + 1] * _col3(Ls[j], top[j], row[j], O, row[j], bot[j]))
            den = torch.sum(Rs[j + 1] * _col3(Ls[j], top[j], row[j], I, row[j], bot[j]))
        else:
            num = 0.0
            for A, B in operator_schmidt(op):
                X = _col3(Ls[j], top[j], row[j], torch.tensor(A, dtype=dt), row[j], bot[j])
                X = _col3(X, top[j + 1], row[j + 1], torch.tensor(B, dtype=dt), row[j + 1], bot[j + 1])
                num = num + torch.sum(Rs[j + 2] * X)
            X = _col3(Ls[j], top[j], row[j], I, row[j], bot[j])
            X = _col3(X, top[j + 1], row[j + 1], I, row[j + 1], bot[j + 1])
            den = torch.sum(Rs[j + 2] * X)
        out.append(num / den)
    return out


def _pair_terms(top, row1, row2, bot, terms_here, d, dt):
    n = len(row1)
    I = torch.eye(d, dtype=dt)
    one = torch.ones((1,) * 6, dtype=dt)
    Ls = [one]
    for j in range(n):
        Ls.append(_norm(_col4(Ls[-1], top[j], row1[j], I, row1[j], row2[j], I, row2[j], bot[j])))
    Rs = [one]
    for j in reversed(range(n)):
        Tp, T1, _, Bt = _mirror3(top[j], row1[j], row1[j], bot[j])
        T2 = row2[j].permute(0, 1, 3, 2, 4)
        Rs.append(_norm(_col4(Rs[-1], Tp, T1, I, T1, T2, I, T2, Bt)))
    Rs = Rs[::-1]
    out = []
    for sites, op in terms_here:
        j = sites[0][1]
        num = 0.0
        for A, B in operator_schmidt(op):
            X = _col4(Ls[j], top[j], row1[j], torch.tensor(A, dtype=dt), row1[j], row2[j],
                      torch.tensor(B, dtype=dt), row2[j], bot[j])
            num = num + torch.sum(Rs[j + 1] * X)
        X = _col4(Ls[j], top[j], row1[j], I, row1[j], row2[j], I, row2[j], bot[j])
        den = torch.sum(Rs[j + 1] * X)
        out.append(num / den)
    return out


def energy(ket, terms, m, p, q, seed):
    """E = sum_t <psi|H_t|psi> / <psi|psi> with cached environments
    (oracle.energy.peps_energy_cached) as a differentiable complex torch scalar.
    The environments are computed in the tensors' own dtype; the strips in
    complex128 (the operators are complex)."""
    nrow, ncol = len(ket), len(ket[0])
    d = ket[0][0].shape[4]
    dt = torch.complex128
    if nrow > 1:
        top_envs, _ = _boundary_pass(ket, TOP, m, p, q, seed)
        bot_envs, _ = _boundary_pass(ket, BOTTOM, m, p, q, seed)
        top_envs = [[S.to(dt) for S in e] for e in top_envs]
        bot_envs = [[S.to(dt) for S in e] for e in bot_envs]
    kn = [[T.to(dt) for T in row] for row in ket]
    triv = [torch.ones((1, 1, 1, 1), dtype=dt) for _ in range(ncol)]
    top_of = lambda i: triv if i == 0 else top_envs[i - 1]
    bot_of = lambda i: triv if i == nrow - 1 else bot_envs[nrow - 2 - i]
    total = 0.0
    for i in range(nrow):
        here = [t for t in terms if all(s[0] == i for s in t[0])]
        if here:
            total = total + sum(_row_terms(top_of(i), kn[i], bot_of(i), here, d, dt))
    for i in range(nrow - 1):
        here = [t for t in terms if len(t[0]) == 2 and t[0][0][0] == i and t[0][1][0] == i + 1]
        if here:
            total = total + sum(_pair_terms(top_of(i), kn[i], kn[i + 1], bot_of(i + 1), here, d, dt))
    return total


def _leaves(ket_np):
    dt = torch.complex128 if np.iscomplexobj(ket_np[0][0]) else torch.float64
    return [[torch.tensor(np.asarray(T), dtype=dt, requires_grad=True) for T in row] for row in ket_np]


def log_norm_grad(ket_np, m, p, q, seed):
    """(log <psi|psi>, gradients as rows of numpy arrays)."""
    ket = _leaves(ket_np)
    L = log_norm(ket, m, p, q, seed)
    L.backward()
    return float(L.detach()), [[T.grad.numpy() for T in row] for row in ket]


def energy_grad(ket_np, terms, m, p, q, seed):
    """(E complex, gradients of Re E as rows of numpy arrays)."""
    ket = _leaves(ket_np)
    E = energy(ket, terms, m, p, q, seed)
    torch.real(E).backward()
    return complex(E.detach()), [[T.grad.numpy() for T in row] for row in ket]


def log_norm_value(ket_np, m, p, q, seed):
    with torch.no_grad():
        dt = torch.complex128 if np.iscomplexobj(ket_np[0][0]) else torch.float64
        return float(log_norm([[torch.tensor(T, dtype=dt) for T in row] for row in ket_np], m, p, q, seed))


def energy_value(ket_np, terms, m, p, q, seed):
    with torch.no_grad():
        dt = torch.complex128 if np.iscomplexobj(ket_np[0][0]) else torch.float64
        return complex(energy([[torch.tensor(T, dtype=dt) for T in row] for row in ket_np], terms, m, p, q, seed))
