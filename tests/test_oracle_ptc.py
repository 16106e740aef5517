"""The parallel-transport network: Neumann-series weights give 1 + kH + k^2 H^2
exactly (ties the layer to the pinned hopping term), gauge equivariance, the
adjoint identity, the weight gradient against central finite differences, and
the identity behind the GPU's folded inference: two linear layers equal
sum_{p,q} T_p K_pq T_q with K_pq = sum_c W2_p^c W1_q^c (its adjoint with
K'_pq = K_{m(q) m(p)}^dagger), and on an odd-site input the odd output keeps
only K_00 and the hop-hop pairs."""
import numpy as np
import pytest

import latgen
from oracle import ptc
from oracle import wilson as W


def _rand_w(rng, cout, cin, scale=0.3):
    return scale * (rng.standard_normal((9, cout, cin, 4, 4)) + 1j * rng.standard_normal((9, cout, cin, 4, 4)))


def test_neumann2():
    cfg = latgen.small_config((4, 2, 2, 4), seed=21)
    U, psi, k = cfg["U"], cfg["b"][0], 0.12
    got = ptc.network(U, ptc.neumann2_weights(k), psi)
    h = W.hop(U, psi)
    want = psi + k * h + k * k * W.hop(U, h)
    assert np.abs(got - want).max() < 1e-13


def test_equivariance():
    dims = (4, 2, 2, 4)
    cfg = latgen.small_config(dims, seed=22)
    U, psi = cfg["U"], cfg["b"][0]
    rng = np.random.default_rng(0)
    ws = [_rand_w(rng, 3, 1), _rand_w(rng, 1, 3)]
    om = latgen.random_su3_field(3, dims)
    Ug = np.empty_like(U)
    for d in range(4):
        Ug[..., d, :, :] = om @ U[..., d, :, :] @ W.dagger3(W.shift_fwd(om, d))
    lhs = ptc.network(Ug, ws, om @ psi)
    rhs = om @ ptc.network(U, ws, psi)
    assert np.abs(lhs - rhs).max() < 1e-13


def test_adjoint_identity():
    cfg = latgen.small_config((4, 2, 2, 4), seed=23, nrhs=4)
    U = cfg["U"]
    rng = np.random.default_rng(1)
    w = _rand_w(rng, 2, 3)
    x = np.stack([cfg["b"][0], cfg["b"][1], cfg["b"][2]])
    y = np.stack([cfg["b"][3], 0.5 * cfg["b"][0]])
    lhs = np.vdot(y, ptc.layer(U, w, x))
    rhs = np.vdot(ptc.layer_adjoint(U, w, y), x)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_wgrad_finite_differences():
    cfg = latgen.small_config((2, 2, 2, 2), seed=24, nrhs=2)
    U = cfg["U"]
    rng = np.random.default_rng(2)
    ws = [_rand_w(rng, 2, 1), _rand_w(rng, 1, 2)]
    src, tgt = cfg["b"][0], cfg["b"][1]
    L0, grads = ptc.loss_and_grad(U, ws, src, tgt)
    h = 1e-6
    for layer in (0, 1):
        for idx in [(0, 0, 0, 1, 2), (3, 0, 0, 0, 0), (8, 0, 1, 3, 3) if layer == 1 else (8, 1, 0, 3, 3)]:
            for part, unit in (("re", 1.0), ("im", 1j)):
                wp = [w.copy() for w in ws]
                wm = [w.copy() for w in ws]
                wp[layer][idx] += unit * h
                wm[layer][idx] -= unit * h
                fd = (ptc.loss_and_grad(U, wp, src, tgt)[0] - ptc.loss_and_grad(U, wm, src, tgt)[0]) / (2 * h)
                G = grads[layer][idx]
                an = 2 * (G.real if part == "re" else G.imag)
                assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (layer, idx, part, fd, an)


def _fold(ws):
    """K[p, q] = sum_c W2[p, 0, c] @ W1[q, c, 0] (4x4 spin matrices)."""
    w1, w2 = ws
    return np.einsum("pcrs,qcst->pqrt", w2[:, 0], w1[:, :, 0])


def _apply_pairs(U, K, v, ps=range(9), qs=range(9)):
    """sum_{p in ps} T_p sum_{q in qs} K[p, q] T_q v."""
    t = {q: ptc.transport(U, v, q) for q in qs}
    out = np.zeros_like(v)
    for p in ps:
        m = sum(t[q] @ K[p, q].T for q in qs)
        out += ptc.transport(U, m, p)
    return out


@pytest.mark.parametrize("hidden", [2, 8])
def test_two_layers_fold_into_path_pairs(hidden):
    dims = (4, 2, 2, 4)
    cfg = latgen.small_config(dims, seed=25, nrhs=1)
    U, v = cfg["U"], cfg["b"][0]
    rng = np.random.default_rng(3)
    ws = [_rand_w(rng, hidden, 1), _rand_w(rng, 1, hidden)]
    K = _fold(ws)
    want = ptc.network(U, ws, v)
    assert np.abs(_apply_pairs(U, K, v) - want).max() < 1e-12 * np.abs(want).max()
    # adjoint: K'[p, q] = K[m(q), m(p)]^dagger
    m = [ptc.mirror(p) for p in range(9)]
    Ka = np.conj(np.swapaxes(K[np.ix_(m, m)].transpose(1, 0, 2, 3), 2, 3))
    want_a = ptc.network_adjoint(U, ws, v)
    assert np.abs(_apply_pairs(U, Ka, v) - want_a).max() < 1e-12 * np.abs(want_a).max()
    # Schur restriction P_o N (0 + v_o): the identity pair on odd sites plus the
    # hop-hop pairs through the even sites; every other pair adds zero
    par = W.parity_field(dims)
    vo = W.project(v, 1)
    want_s = W.project(ptc.network(U, ws, vo), 1)
    hops = range(1, 9)
    got_s = W.project(vo @ K[0, 0].T + _apply_pairs(U, K, vo, hops, hops), 1)
    assert par.any() and np.abs(got_s - want_s).max() < 1e-12 * np.abs(want_s).max()
