"""GPU parity of the QR-SVD two-site update (Alg. 1, Eq. 4) and of batched
TEBD sweeps (Sec. II-D) against the oracle.  Tensors are compared through
gauge-invariant quantities: the kept singular values, the two-site product
over the new bond, and normalised state vectors."""
import numpy as np
import pytest

import synth
from oracle import ite, statevector as sv

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
hp = pytest.importorskip("paper_2006_15234_amd")


@pytest.fixture(scope="module")
def ctx():
    return hp.Context(0)


def dev_lattice(peps):
    return [[torch.from_numpy(np.ascontiguousarray(t)).cuda() for t in row] for row in peps]


def host_lattice(peps):
    return [[t.cpu().numpy() for t in row] for row in peps]


def _pair_product(T1, T2, axis):
    if axis == 0:
        return np.einsum("udlbp,UDbRP->udlpUDRP", T1, T2)
    return np.einsum("ublrp,bDLRP->ulrpDLRP", T1, T2)


@pytest.mark.parametrize("axis", [0, 1])
@pytest.mark.parametrize("D,Dmax", [(2, 2), (2, 4), (3, 3), (4, 4), (4, 8), (8, 8)])
def test_two_site_gate_parity(ctx, axis, D, Dmax):
    nrow, ncol = (3, 4) if axis == 0 else (4, 3)
    peps = synth.random_peps(nrow, ncol, D=D, seed=D * 10 + Dmax)
    rng = np.random.default_rng(D)
    H = rng.standard_normal((4, 4))
    G = synth.bond_gate((H + H.T).reshape(2, 2, 2, 2), 0.3)
    i, j = 1, 1
    i2, j2 = (i, j + 1) if axis == 0 else (i + 1, j)
    T1n, T2n, s = ite.qr_svd_update(peps[i][j], peps[i2][j2], G, axis, Dmax)
    new, sg = hp.apply_two_site_gate(ctx, dev_lattice(peps), i, j, axis,
                                     torch.from_numpy(G).cuda(), Dmax)
    h = host_lattice(new)
    assert h[i][j].shape == T1n.shape and h[i2][j2].shape == T2n.shape
    assert np.max(np.abs(sg.cpu().numpy() - s)) < 1e-12
    pa, pb = _pair_product(h[i][j], h[i2][j2], axis), _pair_product(T1n, T2n, axis)
    assert np.max(np.abs(pa - pb)) < 1e-12 * np.max(np.abs(pb))
    # untouched sites are unchanged
    assert np.array_equal(h[0][0], peps[0][0])


def _tfi_plan_inputs(nrow, ncol, tau, J=1.0, hfield=3.0):
    layers = synth.lattice_bonds(nrow, ncol)
    hams = synth.tfi_bond_hamiltonians(nrow, ncol, J, hfield)
    gates = {b: synth.bond_gate(H, tau) for b, H in hams.items()}
    uniq, index, bond_gate = [], {}, []
    for layer in layers:
        for b in layer:
            key = gates[b].tobytes()
            if key not in index:
                index[key] = len(uniq)
                uniq.append(gates[b])
            bond_gate.append(index[key])
    return layers, gates, np.stack(uniq), bond_gate


def _overlap(a, b):
    return abs(np.vdot(a, b)) / (np.linalg.norm(a) * np.linalg.norm(b))


@pytest.mark.parametrize("shape,Dmax,sweeps", [((2, 2), 8, 3), ((2, 3), 8, 4), ((3, 3), 4, 3),
                                               ((4, 4), 3, 5), ((3, 4), 2, 6)])
@pytest.mark.parametrize("use_graph", [True, False])
def test_ite_sweeps_match_oracle(ctx, shape, Dmax, sweeps, use_graph):
    nrow, ncol = shape
    layers, gates, uniq, bond_gate = _tfi_plan_inputs(nrow, ncol, 0.1)
    peps0 = synth.product_state_peps(nrow, ncol, seed=3)
    ref, _ = ite.ite(peps0, layers, gates, Dmax, sweeps)
    plan = hp.ItePlan(ctx, dev_lattice(peps0), torch.from_numpy(uniq).cuda(), bond_gate, Dmax)
    plan.run(sweeps, use_graph=use_graph)
    got = host_lattice(plan.state())
    plan.close()
    for r in range(nrow):
        for c in range(ncol):
            assert got[r][c].shape == ref[r][c].shape
    ov = _overlap(sv.peps_to_statevector(got).ravel(), sv.peps_to_statevector(ref).ravel())
    assert abs(1 - ov) < 1e-10


def test_ite_graph_replay_is_deterministic(ctx):
    layers, gates, uniq, bond_gate = _tfi_plan_inputs(4, 4, 0.05)
    peps0 = synth.product_state_peps(4, 4, seed=1)
    outs = []
    for use_graph in (True, True, False):
        plan = hp.ItePlan(ctx, dev_lattice(peps0), torch.from_numpy(uniq).cuda(), bond_gate, 4)
        plan.run(3, use_graph=use_graph)
        plan.run(2, use_graph=use_graph)
        outs.append(host_lattice(plan.state()))
        plan.close()
    for o in outs[1:]:
        for r in range(4):
            for c in range(4):
                assert np.array_equal(o[r][c], outs[0][r][c])
