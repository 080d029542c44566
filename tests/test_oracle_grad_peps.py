"""Pins of the contraction-gradient oracle (oracle/grad_peps.py): its forward
values equal the numpy oracle's (oracle.bmps, oracle.energy), and its
gradients equal central finite differences of those values (h = 1e-6,
real and imaginary parts perturbed separately)."""
import numpy as np
import pytest

import synth
from oracle import bmps, energy as oe, grad_peps as gp

torch = pytest.importorskip("torch")

X = np.array([[0, 1], [1, 0]], dtype=complex)
Y = np.array([[0, -1j], [1j, 0]])
Z = np.diag([1.0, -1.0]).astype(complex)


def _terms():
    return [
        (((0, 0),), Z),
        (((1, 2),), X),
        (((1, 1), (1, 2)), (np.kron(Z, Z) + 0.3 * np.kron(Y, Y)).reshape(2, 2, 2, 2)),
        (((0, 1), (1, 1)), np.kron(X, X).reshape(2, 2, 2, 2)),
        (((2, 0), (2, 1)), np.kron(X, Z).reshape(2, 2, 2, 2)),
    ]


@pytest.mark.parametrize("cplx", [False, True])
def test_forward_equals_numpy_oracle(cplx):
    ket = synth.random_peps(3, 4, 2, 2, seed=11, complex_=cplx)
    ln, _ = bmps.peps_norm(ket, 4, 2, 1, 5)
    assert abs(gp.log_norm_value(ket, 4, 2, 1, 5) - ln) < 1e-12
    E, _ = oe.peps_energy_cached(ket, _terms(), 4, 2, 1, 5)
    assert abs(gp.energy_value(ket, _terms(), 4, 2, 1, 5) - E) < 1e-12 * max(1.0, abs(E))


def _fd(f, ket, i, j, idx, cplx, h=1e-6):
    out = 0.0
    for part in ((1.0, 1j) if cplx else (1.0,)):
        vals = []
        for sgn in (1, -1):
            k2 = [[T.copy() for T in row] for row in ket]
            k2[i][j][idx] += sgn * h * part
            vals.append(f(k2))
        out = out + (vals[0] - vals[1]) / (2 * h) * part
    return out


@pytest.mark.parametrize("cplx", [False, True])
def test_log_norm_gradient_finite_differences(cplx):
    ket = synth.random_peps(3, 3, 2, 2, seed=3, complex_=cplx)
    m, p, q, seed = 3, 2, 1, 9
    _, g = gp.log_norm_grad(ket, m, p, q, seed)
    rng = np.random.default_rng(0)
    scale = max(np.max(np.abs(t)) for row in g for t in row)
    for _ in range(10):
        i, j = rng.integers(0, 3, size=2)
        idx = tuple(rng.integers(0, s) for s in ket[i][j].shape)
        fd = _fd(lambda k: gp.log_norm_value(k, m, p, q, seed), ket, i, j, idx, cplx)
        assert abs(fd - g[i][j][idx]) < 1e-6 * scale, (i, j, idx)


@pytest.mark.parametrize("cplx", [False, True])
def test_energy_gradient_finite_differences(cplx):
    ket = synth.random_peps(3, 3, 2, 2, seed=8, complex_=cplx)
    m, p, q, seed = 3, 2, 1, 4
    _, g = gp.energy_grad(ket, _terms(), m, p, q, seed)
    rng = np.random.default_rng(1)
    scale = max(np.max(np.abs(t)) for row in g for t in row)
    for _ in range(10):
        i, j = rng.integers(0, 3, size=2)
        idx = tuple(rng.integers(0, s) for s in ket[i][j].shape)
        fd = _fd(lambda k: gp.energy_value(k, _terms(), m, p, q, seed).real, ket, i, j, idx, cplx)
        assert abs(fd - g[i][j][idx]) < 1e-6 * scale, (i, j, idx)


def test_energy_gradient_scale_invariant():
    """E is invariant under rescaling any one site, so its gradient is orthogonal
    to that site: Re <g_ij, T_ij> = 0 for every site."""
    ket = synth.random_peps(3, 3, 2, 2, seed=2, complex_=True)
    _, g = gp.energy_grad(ket, _terms(), 3, 2, 1, 6)
    for i in range(3):
        for j in range(3):
            assert abs(np.real(np.vdot(g[i][j], ket[i][j]))) < 1e-10 * np.max(np.abs(g[i][j]))
