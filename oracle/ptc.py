"""Parallel-transport convolution (PTC) network, complex128 -- the learned
gauge-covariant preconditioner (an addition to the paper; the layer is the
one of Lehner & Wettig, Phys. Rev. D 108 (2023) 034503).

One layer maps C_in channels of spinor fields to C_out channels:

    psi_out^i(x) = sum_j sum_p W_p^{ij} [T_p psi_in^j](x)

with 9 paths p = 0 (T_0 = 1), +mu (T_{+mu} psi(x) = U_mu(x) psi(x+mu)) and
-mu (T_{-mu} psi(x) = U_mu(x-mu)^dagger psi(x-mu)), mu = x, y, z, t, and
W_p^{ij} a complex 4x4 spin matrix.  Weights have shape (9, C_out, C_in, 4, 4)
with path index order 0, +x, +y, +z, +t, -x, -y, -z, -t.  No nonlinearity.

Since T_{+mu}^dagger = T_{-mu}, the adjoint of a layer (the backward pass for
data) uses the transposed-conjugated weights with mirrored paths.  For a real
loss L of the outputs with g^i = dL/d conj(psi_out^i), the derivative with
respect to the weights is dL/d conj(W_p^{ij}) = sum_{x,c} g^i(x) (T_p psi_in^j)(x)^dagger
(outer product over spin, summed over sites and colour); the gradient with
respect to the real and imaginary parts is twice its real and imaginary part.
"""
import numpy as np

from . import wilson as W

NPATH = 9


def path_dir(p):
    """(mu, sign) of path p >= 1."""
    return (p - 1) % 4, (1 if p <= 4 else -1)


def transport(U, psi, p):
    if p == 0:
        return psi
    mu, sgn = path_dir(p)
    u = U[..., mu, :, :]
    if sgn > 0:
        return u @ W.shift_fwd(psi, mu)
    return W.dagger3(W.shift_bwd(u, mu)) @ W.shift_bwd(psi, mu)


def mirror(p):
    if p == 0:
        return 0
    return p + 4 if p <= 4 else p - 4


def layer(U, w, psi):
    """w: (9, Cout, Cin, 4, 4); psi: (Cin, ...site..., 3, 4) -> (Cout, ...)."""
    cout, cin = w.shape[1], w.shape[2]
    out = np.zeros((cout,) + psi.shape[1:], dtype=np.complex128)
    for p in range(NPATH):
        for j in range(cin):
            tp = transport(U, psi[j], p)
            for i in range(cout):
                out[i] += tp @ w[p, i, j].T
    return out


def layer_adjoint(U, w, g):
    """Adjoint of ``layer`` in its input: (Cout, ...) -> (Cin, ...).
    sum_i sum_p T_p^dagger (W_p^{ij})^dagger g^i."""
    cout, cin = w.shape[1], w.shape[2]
    out = np.zeros((cin,) + g.shape[1:], dtype=np.complex128)
    for p in range(NPATH):
        for j in range(cin):
            acc = np.zeros(g.shape[1:], dtype=np.complex128)
            for i in range(cout):
                acc += g[i] @ np.conj(w[p, i, j])          # spin: (W^dagger) applied = f conj(W)
            out[j] += transport(U, acc, mirror(p))
    return out


def layer_wgrad(U, psi, g):
    """G[p, i, j] = sum_{x,c} g^i(x)[c, :] outer conj((T_p psi^j)(x)[c, :])  (4x4)."""
    cout, cin = g.shape[0], psi.shape[0]
    G = np.zeros((NPATH, cout, cin, 4, 4), dtype=np.complex128)
    for p in range(NPATH):
        for j in range(cin):
            tp = transport(U, psi[j], p).reshape(-1, 4)
            for i in range(cout):
                G[p, i, j] = g[i].reshape(-1, 4).T @ np.conj(tp)
    return G


def network(U, weights, psi):
    """Apply the layers in order to a single field psi (...site..., 3, 4)."""
    h = psi[None]
    for w in weights:
        h = layer(U, w, h)
    return h[0]


def network_adjoint(U, weights, g):
    h = g[None]
    for w in reversed(weights):
        h = layer_adjoint(U, w, h)
    return h[0]


def loss_and_grad(U, weights, src, target):
    """L = ||N(src) - target||^2 / ||target||^2 and dL/d conj(W) per layer."""
    acts = [src[None]]
    for w in weights:
        acts.append(layer(U, w, acts[-1]))
    diff = acts[-1][0] - target
    nt = W.norm2(target)
    L = W.norm2(diff) / nt
    g = (diff / nt)[None]
    grads = [None] * len(weights)
    for k in range(len(weights) - 1, -1, -1):
        grads[k] = layer_wgrad(U, acts[k], g)
        if k > 0:
            g = layer_adjoint(U, weights[k], g)
    return L, grads


def neumann2_weights(kappa, hidden=8):
    """Weights for which the 1 -> hidden -> 1 network equals 1 + kappa H + kappa^2 H^2
    (channel 0 carries psi, channel 1 carries H psi, the rest are zero)."""
    from .gamma import P_MINUS, P_PLUS
    w1 = np.zeros((NPATH, hidden, 1, 4, 4), dtype=np.complex128)
    w2 = np.zeros((NPATH, 1, hidden, 4, 4), dtype=np.complex128)
    w1[0, 0, 0] = np.eye(4)
    for mu in range(4):
        w1[1 + mu, 1, 0] = P_MINUS[mu]
        w1[5 + mu, 1, 0] = P_PLUS[mu]
        w2[1 + mu, 0, 1] = kappa * kappa * P_MINUS[mu]
        w2[5 + mu, 0, 1] = kappa * kappa * P_PLUS[mu]
    w2[0, 0, 0] = np.eye(4)
    w2[0, 0, 1] = kappa * np.eye(4)
    return [w1, w2]
