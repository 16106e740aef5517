"""The parallel-transport network: Neumann-series weights give 1 + kH + k^2 H^2
exactly (ties the layer to the pinned hopping term), gauge equivariance, the
adjoint identity, and the weight gradient against central finite differences."""
import numpy as np

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
