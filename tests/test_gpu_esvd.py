"""GPU parity of einsumsvd (randomized SVD on the implicit zip-up and pair
operators, Alg. 4) against the FP64 CPU oracle on the same seeded inputs and
the same sketch.

Tolerances (normwise, relative to sigma_1): 1e-10 for FP64 / complex128
sketches, 1e-4 for FP32 sketches.  The factor product U diag(s) V^* is
compared entrywise; U is checked to be an isometry."""
import numpy as np
import pytest

import synth
from oracle import rsvd
from oracle.network import pair_operator, zipup_operator
from oracle.sketch import sketch as oracle_sketch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def _rand(rng, shape, cplx):
    x = rng.standard_normal(shape)
    if cplx:
        x = x + 1j * rng.standard_normal(shape)
    return x / np.linalg.norm(x)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def test_sketch_bitwise(ctx):
    g = hp.sketch(ctx, 1000, 37, batch=3, seed=12345, stream_id=77).cpu().numpy()
    for b in range(3):
        ref = oracle_sketch(12345, 77 + b, 1000, 37)
        assert np.array_equal(g[b], ref)
    g32 = hp.sketch(ctx, 300, 20, seed=5, stream_id=9, precision="f32").cpu().numpy()
    assert np.array_equal(g32[0], oracle_sketch(5, 9, 300, 20).astype(np.float32))


def _check(U, s, R, Uo, so, Vho, tol, absorb):
    s1 = so[0]
    assert np.max(np.abs(s - so)) <= tol * s1
    if absorb == hp.ABSORB_CARRY:
        Vh = R * (s1 / s)[:, None]
    elif absorb == hp.ABSORB_RIGHT:
        Vh = R / s[:, None]
    else:
        Vh = R
    prod = (U * s) @ Vh
    ref = (Uo * so) @ Vho
    assert np.max(np.abs(prod - ref)) <= tol * s1 * 10
    mp = U.shape[1]
    assert np.max(np.abs(U.conj().T @ U - np.eye(mp))) < (1e-11 if tol < 1e-8 else 1e-5)


ZIP_CASES = [
    # a, x, b, h, u, c, y, g, d, m, p, q, cplx
    (1, 2, 1, 2, 2, 3, 2, 2, 2, 4, 4, 1, False),      # first column: a = 1, square-ish
    (3, 2, 2, 2, 2, 3, 2, 2, 2, 5, 3, 2, False),
    (5, 3, 4, 2, 3, 5, 3, 1, 2, 7, 5, 1, False),      # g = 1 (last-column-like)
    (4, 2, 3, 3, 2, 4, 2, 2, 2, 6, 2, 0, True),       # complex
    (7, 3, 5, 3, 3, 6, 3, 2, 2, 20, 8, 2, False),     # several tiles, ragged
    (6, 2, 5, 2, 2, 5, 2, 2, 2, 12, 4, 1, True),
]


@pytest.mark.parametrize("case", ZIP_CASES)
@pytest.mark.parametrize("absorb", [0, 1, 2])
def test_zipup_parity(ctx, case, absorb):
    a, x, b, h, u, c, y, g, d, m, p, q, cplx = case
    rng = np.random.default_rng(hash(case) % 2 ** 32)
    B = 2
    Vs = [_rand(rng, (a, x, x, b, h, h), cplx) for _ in range(B)]
    Ss = [_rand(rng, (b, u, u, c), cplx) for _ in range(B)]
    Ts = [_rand(rng, (u, y, h, g, d), cplx) for _ in range(B)]
    Bs = [_rand(rng, (u, y, h, g, d), cplx) for _ in range(B)]
    seed, sid = 42, 1000
    ls = torch.zeros(B, dtype=torch.float64, device="cuda")
    U, s, R = hp.einsumsvd_zipup(ctx, _dev(np.stack(Vs)), _dev(np.stack(Ss)), _dev(np.stack(Ts)),
                                 _dev(np.stack(Bs)), rank=m, oversample=p, power_iters=q, seed=seed,
                                 stream_id=sid, absorb=absorb, log_scale=ls)
    U, s, R, ls = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy(), ls.cpu().numpy()
    for i in range(B):
        op = zipup_operator(Vs[i], Ss[i], Ts[i], Bs[i])
        k = rsvd.sketch_width(m, p, op.n_rows, op.n_cols)
        om = oracle_sketch(seed, sid + i, op.n_cols, k)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, m, q, om)
        mp = so.shape[0]
        _check(U[i].reshape(-1, mp), s[i], R[i].reshape(mp, -1), Uo, so, Vho, 1e-10, absorb)
        if absorb == hp.ABSORB_CARRY:
            assert abs(ls[i] - np.log(so[0])) < 1e-12
        else:
            assert ls[i] == 0.0


def test_zipup_exact_regime_equals_definition(ctx):
    """k = min(rows, cols): the GPU result is the exact truncated SVD."""
    rng = np.random.default_rng(3)
    a, x, b, h, u, c, y, g, d = 2, 2, 2, 2, 2, 2, 2, 1, 2
    V = _rand(rng, (1, a, x, x, b, h, h), False)
    S = _rand(rng, (1, b, u, u, c), False)
    T = _rand(rng, (1, u, y, h, g, d), False)
    U, s, R = hp.einsumsvd_zipup(ctx, _dev(V), _dev(S), _dev(T), None, rank=8, oversample=0,
                                 power_iters=0, absorb=hp.ABSORB_RIGHT)
    A = zipup_operator(V[0], S[0], T[0], T[0]).explicit()
    ref = np.linalg.svd(A, compute_uv=False)
    s = s.cpu().numpy()[0]
    assert np.allclose(s, ref[:8], atol=1e-13 * ref[0])
    prod = U.cpu().numpy()[0].reshape(8, 8) @ R.cpu().numpy()[0].reshape(8, 8)
    assert np.max(np.abs(prod - A)) < 1e-13 * ref[0] * 10


PAIR_CASES = [(6, 2, 2, 8, 4, 1), (8, 3, 2, 10, 6, 2), (12, 3, 2, 16, 8, 2)]


@pytest.mark.parametrize("case", PAIR_CASES)
@pytest.mark.parametrize("cplx", [False, True])
def test_pair_parity(ctx, case, cplx):
    m, D, d, rank, p, q = case
    B = 3
    inst = [synth.pair_instance(m, D, d, seed=7, instance=i, complex_=cplx) for i in range(B)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                power_iters=q, seed=3, stream_id=11, absorb=hp.ABSORB_NONE)
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    for i in range(B):
        op = pair_operator(*inst[i])
        k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
        om = oracle_sketch(3, 11 + i, op.n_cols, k)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        mp = so.shape[0]
        _check(U[i].reshape(-1, mp), s[i], R[i].reshape(mp, -1), Uo, so, Vho, 1e-10, hp.ABSORB_NONE)


def test_pair_fp32_sketch(ctx):
    m, D, d, rank, p, q = 12, 3, 2, 16, 8, 3
    inst = [synth.pair_instance(m, D, d, seed=9, instance=i) for i in range(2)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                power_iters=q, seed=1, stream_id=5, precision="f32",
                                absorb=hp.ABSORB_NONE)
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    for i in range(2):
        op = pair_operator(*inst[i])
        k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
        om = oracle_sketch(1, 5 + i, op.n_cols, k)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        assert np.max(np.abs(s[i] - so)) <= 1e-4 * so[0]
        prod = (U[i].reshape(-1, rank) * s[i]) @ R[i].reshape(rank, -1)
        assert np.max(np.abs(prod - (Uo * so) @ Vho)) <= 1e-4 * so[0] * 10


@pytest.mark.parametrize("shape", [(12, 3, 2, 16, 8, 3), (20, 4, 2, 24, 8, 2)])
def test_pair_bf16_sketch(ctx, shape):
    """BF16 operator applications (FP32 accumulation, FP64 factorizations): singular values
    normwise within 3e-2 of the FP64 oracle on the same (unrounded) sketch."""
    m, D, d, rank, p, q = shape
    inst = [synth.pair_instance(m, D, d, seed=9, instance=i) for i in range(2)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                power_iters=q, seed=1, stream_id=5, precision="bf16",
                                absorb=hp.ABSORB_NONE)
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    for i in range(2):
        op = pair_operator(*inst[i])
        k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
        om = oracle_sketch(1, 5 + i, op.n_cols, k)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        assert np.max(np.abs(s[i] - so)) <= 3e-2 * so[0]
        # the left factor is an isometry to FP64 accuracy (orthogonalization stays FP64)
        Ui = U[i].reshape(-1, rank)
        assert np.max(np.abs(Ui.T @ Ui - np.eye(rank))) < 1e-10


@pytest.mark.parametrize("tile", range(15))
@pytest.mark.parametrize("precision,tol", [("f32", 1e-4), ("bf16", 3e-2)])
def test_pair_mixed_every_tile(ctx, tile, precision, tol):
    """Every GEMM tile shape forced on every product of an FP32 and a BF16 einsumsvd (BF16
    takes 32-deep K-steps and maps the shapes of more than 8 MFMA tiles per wavefront to
    128 x 64): singular values within the precision's tolerance of the FP64 oracle."""
    m, D, d, rank, p, q = 20, 4, 2, 24, 8, 2
    inst = [synth.pair_instance(m, D, d, seed=11, instance=i) for i in range(2)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    try:
        ctx.check(ctx.lib.hpeps_test_gemm_variant(ctx.h, tile, 2 if precision == "bf16" else 1, 0))
        U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                    power_iters=q, seed=1, stream_id=5, precision=precision,
                                    absorb=hp.ABSORB_NONE)
        s = s.cpu().numpy()
    finally:
        ctx.check(ctx.lib.hpeps_test_gemm_variant(ctx.h, -1, 1, 0))
    for i in range(2):
        op = pair_operator(*inst[i])
        k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
        om = oracle_sketch(1, 5 + i, op.n_cols, k)
        _, so, _ = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        assert np.max(np.abs(s[i] - so)) <= tol * so[0]


def test_pair_full_size_bf16(ctx):
    """The benchmarked configuration in BF16: instances 0 and 63, singular values normwise
    within 3e-2 of the FP64 oracle."""
    m, D, d, rank, p, q, B = 36, 6, 2, 36, 8, 2, 64
    inst = [synth.pair_instance(m, D, d, seed=0, instance=i) for i in range(B)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                power_iters=q, seed=0, stream_id=1, precision="bf16",
                                absorb=hp.ABSORB_NONE)
    s = s.cpu().numpy()
    for i in (0, B - 1):
        op = pair_operator(*inst[i])
        om = oracle_sketch(0, 1 + i, op.n_cols, rank + p)
        _, so, _ = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        assert np.max(np.abs(s[i] - so)) <= 3e-2 * so[0]


def test_pair_full_size_sampled(ctx):
    """The benchmarked configuration (m=36, D=6, d=2, rank 36, p=8, q=2, 64
    instances): instances 0 and 63 against the oracle."""
    m, D, d, rank, p, q, B = 36, 6, 2, 36, 8, 2, 64
    inst = [synth.pair_instance(m, D, d, seed=0, instance=i) for i in range(B)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                power_iters=q, seed=0, stream_id=1, absorb=hp.ABSORB_NONE)
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    for i in (0, B - 1):
        op = pair_operator(*inst[i])
        om = oracle_sketch(0, 1 + i, op.n_cols, rank + p)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        _check(U[i].reshape(-1, rank), s[i], R[i].reshape(rank, -1), Uo, so, Vho, 1e-10,
               hp.ABSORB_NONE)


def test_errors_are_reported(ctx):
    V = torch.zeros((1, 1, 2, 2, 1, 2, 2), dtype=torch.float64, device="cuda")
    S = torch.zeros((1, 1, 2, 2, 1), dtype=torch.float64, device="cuda")
    T = torch.zeros((1, 2, 2, 2, 1, 2), dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HpepsError) as e:
        hp.einsumsvd_zipup(ctx, V, S, T, rank=0)
    assert e.value.code == 1
    big = torch.zeros((1, 200, 2, 2, 1, 2, 2), dtype=torch.float64, device="cuda")
    S2 = torch.zeros((1, 1, 2, 2, 100), dtype=torch.float64, device="cuda")
    with pytest.raises(hp.HpepsError) as e:  # rows 800, cols 400: k = 150 > 128
        hp.einsumsvd_zipup(ctx, big, S2, T, rank=150)
    assert e.value.code == 2


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("prec,cplx", [("f64", False), ("f64", True), ("f32", False), ("bf16", False)])
def test_pair_both_contraction_orders(ctx, order, prec, cplx):
    """The pair einsumsvd with each contraction order of the operator's middle stages
    forced, against the FP64 oracle (1e-10 FP64, 1e-4 FP32, 3e-2 BF16)."""
    m, D, d, rank, p, q = 12, 3, 2, 16, 8, 2
    B = 2
    inst = [synth.pair_instance(m, D, d, seed=19, instance=i, complex_=cplx) for i in range(B)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    ctx.check(ctx.lib.hpeps_test_zip_order(ctx.h, order))
    try:
        U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                    power_iters=q, seed=4, stream_id=8, precision=prec,
                                    absorb=hp.ABSORB_NONE)
    finally:
        ctx.check(ctx.lib.hpeps_test_zip_order(ctx.h, 0))
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    tol = {"f64": 1e-10, "f32": 1e-4, "bf16": 3e-2}[prec]
    for i in range(B):
        op = pair_operator(*inst[i])
        k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
        om = oracle_sketch(4, 8 + i, op.n_cols, k)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        if prec == "f64":
            _check(U[i].reshape(-1, rank), s[i], R[i].reshape(rank, -1), Uo, so, Vho, tol,
                   hp.ABSORB_NONE)
        else:
            assert np.max(np.abs(s[i] - so)) <= tol * so[0]


@pytest.mark.parametrize("order", [1, 2])
def test_zipup_both_contraction_orders(ctx, order):
    """A general zip-up einsumsvd (every leg > 1, complex) with each order forced."""
    a, x, b, h, u, c, y, g, d = 4, 2, 3, 2, 2, 3, 2, 2, 2
    rng = np.random.default_rng(5)
    V = _rand(rng, (a, x, x, b, h, h), True)
    S = _rand(rng, (b, u, u, c), True)
    T = _rand(rng, (u, y, h, g, d), True)
    Bra = _rand(rng, (u, y, h, g, d), True)
    rank, p, q = 6, 3, 1
    ctx.check(ctx.lib.hpeps_test_zip_order(ctx.h, order))
    try:
        U, s, R = hp.einsumsvd_zipup(ctx, _dev(V[None]), _dev(S[None]), _dev(T[None]),
                                     _dev(Bra[None]), rank=rank, oversample=p, power_iters=q,
                                     seed=2, stream_id=3, absorb=hp.ABSORB_NONE)
    finally:
        ctx.check(ctx.lib.hpeps_test_zip_order(ctx.h, 0))
    op = zipup_operator(V, S, T, Bra)
    k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
    Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q,
                                      oracle_sketch(2, 3, op.n_cols, k))
    U, s, R = U.cpu().numpy()[0], s.cpu().numpy()[0], R.cpu().numpy()[0]
    _check(U.reshape(-1, rank), s, R.reshape(rank, -1), Uo, so, Vho, 1e-10, hp.ABSORB_NONE)
