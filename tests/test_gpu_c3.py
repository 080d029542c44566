"""GPU parity at the size of the 12 x 12, D = 10, m = 100 boundary contraction (the
mixed-precision norm workload) and of the norm at D >= 6, m >= 36, against the oracle: one
bulk zip-up einsumsvd of that contraction at full size (a 10^4 x 10^6 implicit operator,
k = 108, so the k > 64 Cholesky, Jacobi and orthogonalization paths run on real zip-up
panels) in FP64 (1e-10), FP32 (1e-4) and BF16 (3e-2) operator applications, the norm of a
6 x 6, D = 6 lattice at m = 36, and the pair einsumsvd of the benchmark at full size with
FP32 applications."""
import numpy as np
import pytest

import synth
from oracle import bmps, rsvd
from oracle.network import pair_operator, zipup_operator
from oracle.sketch import sketch as oracle_sketch

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _unit(rng, shape):
    x = rng.standard_normal(shape)
    return x / np.linalg.norm(x)


def test_c3_bulk_einsumsvd_full_size(ctx):
    """A bulk column of the 12 x 12, D = 10, m = 100 norm: carry V [100,10,10,100,10,10],
    boundary tensor S [100,10,10,100], site T [10,10,10,10,2] with its conjugate as the bra
    layer; rank 100, oversampling 8, 1 power iteration.  FP64: singular values normwise at
    1e-10 and U Sigma V^* on three random probe vectors at 1e-10 of its norm; U an isometry.
    FP32 and BF16 operator applications (FP64 factorizations) against the same FP64 oracle:
    singular values normwise at 1e-4 and 3e-2."""
    D, m, d, rank, p, q, seed, sid = 10, 100, 2, 100, 8, 1, 3, 11
    rng = np.random.default_rng(2024)
    V = _unit(rng, (m, D, D, m, D, D))
    S = _unit(rng, (m, D, D, m))
    T = _unit(rng, (D, D, D, D, d))
    op = zipup_operator(V, S, T, T)
    assert (op.n_rows, op.n_cols) == (10 ** 4, 10 ** 6)
    k = rsvd.sketch_width(rank, p, op.n_rows, op.n_cols)
    assert k == 108
    Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q,
                                      oracle_sketch(seed, sid, op.n_cols, k))
    dv = [_dev(t[None]) for t in (V, S, T)]
    probes = rng.standard_normal((op.n_cols, 3))
    ref = (Uo * so) @ (Vho @ probes)
    for prec, tol in (("f64", 1e-10), ("f32", 1e-4), ("bf16", 3e-2)):
        U, s, R = hp.einsumsvd_zipup(ctx, *dv, rank=rank, oversample=p, power_iters=q, seed=seed,
                                     stream_id=sid, precision=prec, absorb=hp.ABSORB_NONE)
        s = s[0].cpu().numpy()
        assert np.max(np.abs(s - so)) <= tol * so[0], prec
        if prec == "f64":
            Um = U[0].cpu().numpy().reshape(op.n_rows, rank)
            Rm = R[0].cpu().numpy().reshape(rank, op.n_cols)
            assert np.max(np.abs(Um.T @ Um - np.eye(rank))) < 1e-12
            got = (Um * s) @ (Rm @ probes)
            assert np.max(np.abs(got - ref)) <= 1e-10 * np.max(np.abs(ref))
        del U, R


@pytest.mark.parametrize("prec,q,tol", [("f64", 1, 1e-10), ("f32", 2, 1e-4), ("bf16", 2, 3e-2)])
def test_norm_d6_m36(ctx, prec, q, tol):
    """<psi|psi> of a 6 x 6, D = 6 lattice (iid N(0,1) sites, each normalised; double-layer
    bond 36) by the boundary MPS at m = 36, p = 8 (four zip-up rows of truncating
    einsumsvds, 1296 x 46656 operators in the bulk) against the oracle's Alg. 2: |d log N|
    within 1e-10 (FP64), 1e-4 (FP32 applications) and 3e-2 (BF16 applications), the mixed
    forms with the extra power iteration on both sides."""
    peps = synth.random_peps(6, 6, D=6, seed=1)
    ln_ref, ph_ref = bmps.peps_norm(peps, 36, 8, q, 0)
    dev = [[_dev(t) for t in row] for row in peps]
    ln, ph = hp.peps_norm(ctx, dev, rank=36, oversample=8, power_iters=q, seed=0, precision=prec)
    bound = tol * max(1.0, abs(ln_ref)) if prec == "f64" else tol
    assert abs(ln - ln_ref) <= bound
    assert abs(ph - ph_ref) <= 1e-10


def test_pair_full_size_fp32(ctx):
    """The benchmarked pair einsumsvd (m = 36, D = 6, d = 2, rank 36, p = 8, q = 2, 64
    instances) with FP32 operator applications: instances 0 and 63 against the FP64
    oracle, singular values normwise within 1e-4 and U Sigma V^* within 1e-4 of sigma_1."""
    m, D, d, rank, p, q, B = 36, 6, 2, 36, 8, 2, 64
    inst = [synth.pair_instance(m, D, d, seed=0, instance=i) for i in range(B)]
    st = [np.stack([t[j] for t in inst]) for j in range(4)]
    U, s, R = hp.einsumsvd_pair(ctx, *[_dev(t) for t in st], rank=rank, oversample=p,
                                power_iters=q, seed=0, stream_id=1, precision="f32",
                                absorb=hp.ABSORB_NONE)
    U, s, R = U.cpu().numpy(), s.cpu().numpy(), R.cpu().numpy()
    for i in (0, B - 1):
        op = pair_operator(*inst[i])
        om = oracle_sketch(0, 1 + i, op.n_cols, rank + p)
        Uo, so, Vho = rsvd.randomized_svd(op.apply, op.apply_adj, op.n_rows, op.n_cols, rank, q, om)
        assert np.max(np.abs(s[i] - so)) <= 1e-4 * so[0]
        prod = (U[i].reshape(-1, rank) * s[i]) @ R[i].reshape(rank, -1)
        assert np.max(np.abs(prod - (Uo * so) @ Vho)) <= 1e-4 * so[0]
