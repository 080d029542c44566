"""GPU parity of the batched network einsumsvd (hpeps_einsumsvd_batched): every
operand carries a leading instance dimension and instance b draws its sketch
from stream stream_id + b.  Each instance is compared with the oracle's Alg. 4
on that instance's explicit matrix with that sketch (1e-10), with the single
network call on the same instance, and, on the zip-up network, with the
specialised batched zip-up call."""
import numpy as np
import pytest

from oracle import rsvd
from oracle.sketch import sketch as oracle_sketch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rand(rng, shape, cplx):
    x = rng.standard_normal(shape)
    if cplx:
        x = x + 1j * rng.standard_normal(shape)
    return x / np.linalg.norm(x)


def _product(U, s, R, absorb, s1=None):
    mp = s.shape[0]
    U = U.reshape(-1, mp)
    R = R.reshape(mp, -1)
    if absorb == hp.ABSORB_NONE:
        R = s[:, None] * R
    elif absorb == hp.ABSORB_CARRY:
        R = s1 * R
    return U @ R


@pytest.mark.parametrize("cplx,absorb", [(False, hp.ABSORB_NONE), (True, hp.ABSORB_NONE),
                                         (False, hp.ABSORB_CARRY), (True, hp.ABSORB_RIGHT)])
def test_batched_network_vs_oracle(ctx, cplx, absorb):
    """A[a,b,c] B[c,d,e] conj(C[e,f,a]) read as ((b,d), f) for 5 instances; B is a transposed
    view of a batched array, so its instance stride is not the row-major one of its legs."""
    rng = np.random.default_rng(31)
    nb = 5
    da, db, dc, dd, de, df = 3, 6, 4, 5, 3, 26
    A = np.stack([_rand(rng, (da, db, dc), cplx) for _ in range(nb)])
    Bt = np.stack([_rand(rng, (de, dd, dc), cplx) for _ in range(nb)])   # [n,e,d,c]
    Cc = np.stack([_rand(rng, (de, df, da), cplx) for _ in range(nb)])
    rank, p, q, seed, sid = 8, 5, 2, 9, 40
    ls = torch.zeros(nb, dtype=torch.float64, device="cuda")
    U, s, R = hp.einsumsvd_batched(ctx, "abc,cde,efa->bd|f", _dev(A), _dev(Bt).permute(0, 3, 2, 1), _dev(Cc),
                                   conj=[False, False, True], rank=rank, oversample=p, power_iters=q,
                                   seed=seed, stream_id=sid, absorb=absorb, log_scale=ls)
    assert tuple(U.shape) == (nb, db, dd, rank) and tuple(R.shape) == (nb, rank, df)
    s = s.cpu().numpy()
    U = U.cpu().numpy()
    R = R.cpu().numpy()
    lsv = ls.cpu().numpy()
    for b in range(nb):
        M = np.einsum("abc,cde,efa->bdf", A[b], Bt[b].transpose(2, 1, 0), Cc[b].conj()).reshape(db * dd, df)
        k = rsvd.sketch_width(rank, p, M.shape[0], M.shape[1])
        Uo, so, Vho = rsvd.randomized_svd(lambda X: M @ X, lambda Y: M.conj().T @ Y, M.shape[0], M.shape[1],
                                          rank, q, oracle_sketch(seed, sid + b, M.shape[1], k))
        assert np.max(np.abs(s[b] - so)) <= 1e-10 * so[0], b
        if absorb == hp.ABSORB_RIGHT:
            P = U[b].reshape(-1, rank) @ R[b].reshape(rank, -1)
        else:
            P = _product(U[b], s[b], R[b], absorb, s1=so[0])
        assert np.max(np.abs(P - (Uo * so) @ Vho)) <= 1e-9 * so[0], b
        if absorb == hp.ABSORB_CARRY:
            assert abs(lsv[b] - np.log(so[0])) < 1e-12, b


@pytest.mark.parametrize("cplx", [False, True])
def test_batched_equals_single_calls(ctx, cplx):
    """Instance b of the batched call is the single call on instance b with stream_id + b."""
    rng = np.random.default_rng(32)
    nb = 3
    X = np.stack([_rand(rng, (7, 9, 4), cplx) for _ in range(nb)])
    Y = np.stack([_rand(rng, (4, 8, 11), cplx) for _ in range(nb)])
    kw = dict(rank=10, oversample=4, power_iters=1, seed=2, absorb=hp.ABSORB_NONE)
    dX, dY = _dev(X), _dev(Y)
    U, s, R = hp.einsumsvd_batched(ctx, "abc,cde->ad|be", dX, dY, stream_id=100, **kw)
    for b in range(nb):
        U1, s1, R1 = hp.einsumsvd(ctx, "abc,cde->ad|be", dX[b], dY[b], stream_id=100 + b, **kw)
        s1 = s1.cpu().numpy()
        assert np.max(np.abs(s[b].cpu().numpy() - s1)) <= 1e-12 * s1[0]
        P1 = _product(U1.cpu().numpy(), s1, R1.cpu().numpy(), hp.ABSORB_NONE)
        P = _product(U[b].cpu().numpy(), s1, R[b].cpu().numpy(), hp.ABSORB_NONE)
        assert np.max(np.abs(P - P1)) <= 1e-12 * s1[0]


def test_batched_zipup_network_equals_zipup_call(ctx):
    """The zip-up network of Alg. 3 over 4 instances, large enough for several GEMM tiles
    per product: the same factors as the specialised batched zip-up call."""
    a, x, b, h, u, c, y, g, d = 12, 3, 6, 3, 3, 12, 3, 3, 2
    rng = np.random.default_rng(33)
    nb = 4
    V = np.stack([_rand(rng, (a, x, x, b, h, h), True) for _ in range(nb)])
    S = np.stack([_rand(rng, (b, u, u, c), True) for _ in range(nb)])
    T = np.stack([_rand(rng, (u, y, h, g, d), True) for _ in range(nb)])
    Bra = np.stack([_rand(rng, (u, y, h, g, d), True) for _ in range(nb)])
    kw = dict(rank=24, oversample=8, power_iters=1, seed=7, stream_id=11, absorb=hp.ABSORB_RIGHT)
    ops = [_dev(V), _dev(S), _dev(T), _dev(Bra)]
    U0, s0, R0 = hp.einsumsvd_zipup(ctx, *ops, **kw)
    U, s, R = hp.einsumsvd_batched(ctx, "axXbhH,buUc,uyhgp,UYHGp->axX|yYcgG", *ops,
                                   conj=[False, False, False, True], **kw)
    for i in range(nb):
        si = s0[i].cpu().numpy()
        assert np.max(np.abs(s[i].cpu().numpy() - si)) <= 1e-10 * si[0], i
        P0 = _product(U0[i].cpu().numpy(), si, R0[i].cpu().numpy(), hp.ABSORB_RIGHT)
        P = _product(U[i].cpu().numpy(), si, R[i].cpu().numpy(), hp.ABSORB_RIGHT)
        assert np.max(np.abs(P - P0)) <= 1e-10 * si[0], i


def test_batched_explicit_method(ctx):
    """method="explicit" (BMPS: the contracted matrix and its dense truncated SVD) per
    instance: the singular values and the best rank-m approximation of each instance."""
    rng = np.random.default_rng(34)
    nb, rank = 3, 6
    A = np.stack([_rand(rng, (5, 4, 6), False) for _ in range(nb)])
    B = np.stack([_rand(rng, (6, 7, 3), False) for _ in range(nb)])
    U, s, R = hp.einsumsvd_batched(ctx, "abc,cde->ab|de", _dev(A), _dev(B), rank=rank,
                                   absorb=hp.ABSORB_RIGHT, method="explicit")
    for b in range(nb):
        M = np.einsum("abc,cde->abde", A[b], B[b]).reshape(20, 21)
        Ue, se, Vhe = np.linalg.svd(M)
        assert np.max(np.abs(s[b].cpu().numpy() - se[:rank])) <= 1e-12 * se[0], b
        P = U[b].cpu().numpy().reshape(-1, rank) @ R[b].cpu().numpy().reshape(rank, -1)
        assert np.max(np.abs(P - (Ue[:, :rank] * se[:rank]) @ Vhe[:rank])) <= 1e-11 * se[0], b


def test_batched_layout_errors(ctx):
    """Instances must be disjoint (batch stride at least one instance) and agree on the
    batch count; batch < 1 is rejected."""
    X = torch.zeros((4, 5), dtype=torch.float64, device="cuda")
    Y = torch.zeros((3, 5, 6), dtype=torch.float64, device="cuda")
    with pytest.raises(Exception):   # stride-0 broadcast: overlapping instances
        hp.einsumsvd_batched(ctx, "ab,bc->a|c", X.expand(3, 4, 5), Y, rank=2)
    with pytest.raises(Exception):   # the batch dimension is not the outermost one
        Z = torch.zeros((4, 3, 5), dtype=torch.float64, device="cuda").permute(1, 0, 2)
        hp.einsumsvd_batched(ctx, "ab,bc->a|c", Z, Y, rank=2)
    with pytest.raises(Exception):   # batch counts differ
        hp.einsumsvd_batched(ctx, "ab,bc->a|c", torch.zeros((2, 4, 5), dtype=torch.float64, device="cuda"),
                             Y, rank=2)
    from paper_2006_15234_amd import _ffi
    import ctypes as C
    descs = (_ffi.Tensor * 2)(*[hp.api._tensor_desc(t, False, "t") for t in (X[None], Y[:1])])
    o = hp.make_opts(2, 0)
    out = torch.zeros(64, dtype=torch.float64, device="cuda")
    st = ctx.lib.hpeps_einsumsvd_batched(ctx.h, hp.F64, 0, b"ab,bc->a|c", 2, descs, C.byref(o),
                                         hp.ABSORB_NONE, out.data_ptr(), None, out.data_ptr(), None)
    assert st != 0


def test_batched_pair_network_full_size(ctx):
    """The benchmarked configuration (pair network m=36, D=6, d=2, rank 36, p=8, q=2, 64
    instances) through the batched network call: every instance's singular values and
    factor product equal the specialised batched pair call (parity-tested against the
    oracle) at 1e-10 relative to sigma_1."""
    import synth
    m, D, d, rank, p, q, B = 36, 6, 2, 36, 8, 2, 64
    inst = [synth.pair_instance(m, D, d, seed=0, instance=i) for i in range(B)]
    st = [_dev(np.stack([x[t] for x in inst])) for t in range(4)]
    kw = dict(rank=rank, oversample=p, power_iters=q, seed=0, stream_id=1, absorb=hp.ABSORB_RIGHT)
    U0, s0, R0 = hp.einsumsvd_pair(ctx, *st, **kw)
    t1 = st[2][:, :, :, 0]           # [B,u,x,h,p] strided view
    t2 = st[3][:, :, :, :, 0]        # [B,v,y,h,q] strided view
    U, s, R = hp.einsumsvd_batched(ctx, "auUb,bvVc,uxhp,UXHp,vyhq,VYHq->axX|yYc", st[0], st[1], t1, t1, t2, t2,
                                   conj=[False, False, False, True, False, True], **kw)
    s0 = s0.cpu().numpy()
    s = s.cpu().numpy()
    assert np.max(np.abs(s - s0) / s0[:, :1]) <= 1e-10
    for i in (0, 17, 63):
        P0 = _product(U0[i].cpu().numpy(), s0[i], R0[i].cpu().numpy(), hp.ABSORB_RIGHT)
        P = _product(U[i].cpu().numpy(), s0[i], R[i].cpu().numpy(), hp.ABSORB_RIGHT)
        assert np.max(np.abs(P - P0)) <= 1e-10 * s0[i, 0], i
