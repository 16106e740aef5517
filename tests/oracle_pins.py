"""Pins of the oracle's Dirac operator against facts that do not depend on the
oracle's own code: the free-field plane-wave spectrum, a constant U(1)
background, gauge covariance, gamma_5-hermiticity and translation invariance.
Each returns a maximum error; the tests and the planted-mistake test use them."""
import numpy as np

import latgen
from oracle import wilson as W
from oracle.gamma import GAMMA, GAMMA5

ID4 = np.eye(4)


def coords(dims):
    lx, ly, lz, lt = dims
    t, z, y, x = np.meshgrid(np.arange(lt), np.arange(lz), np.arange(ly), np.arange(lx), indexing="ij")
    return x, y, z, t


def momentum_D(p, kappa, mu):
    """D(p) = (1 - 2 kappa sum cos p) + 2 i kappa sum gamma_mu sin p_mu + 2 i kappa mu gamma_5."""
    m = (1 - 2 * kappa * np.sum(np.cos(p))) * ID4 + 2j * kappa * mu * GAMMA5
    for d in range(4):
        m = m + 2j * kappa * np.sin(p[d]) * GAMMA[d]
    return m


def pin_free_field(dims=(4, 2, 6, 4), kappa=0.13, mu=0.05, theta=(0, 0, 0, 0), seed=0):
    """D on a plane wave e^{i p.x} chi, with unit links times constant phases
    e^{i theta_mu}: the result is e^{i p.x} D(p + theta) chi."""
    lx, ly, lz, lt = dims
    U = np.zeros((lt, lz, ly, lx, 4, 3, 3), dtype=complex)
    for d in range(4):
        U[..., d, :, :] = np.exp(1j * theta[d]) * np.eye(3)
    x = coords(dims)
    rng = np.random.default_rng(seed)
    err = 0.0
    for n in [(0, 0, 0, 0), (1, 0, 0, 0), (0, 1, 0, 0), (0, 0, 1, 0), (0, 0, 0, 1), (1, 1, 2, 3), (3, 1, 5, 2)]:
        p = np.array([2 * np.pi * n[d] / dims[d] for d in range(4)])
        chi = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
        phase = np.exp(1j * sum(p[d] * x[d] for d in range(4)))
        psi = phase[..., None, None] * chi
        got = W.apply_D(U, kappa, mu, psi)
        want = phase[..., None, None] * (chi @ momentum_D(p + np.array(theta), kappa, mu).T)
        err = max(err, np.abs(got - want).max())
    return err


def pin_covariance(dims=(4, 2, 2, 4), seed=1, kappa=0.12, mu=0.07):
    cfg = latgen.small_config(dims, seed=seed)
    U, psi = cfg["U"], cfg["b"][0]
    om = latgen.random_su3_field(seed, dims)
    Ug = np.empty_like(U)
    for d in range(4):
        Ug[..., d, :, :] = om @ U[..., d, :, :] @ W.dagger3(W.shift_fwd(om, d))
    lhs = W.apply_D(Ug, kappa, mu, om @ psi)
    rhs = om @ W.apply_D(U, kappa, mu, psi)
    return np.abs(lhs - rhs).max()


def pin_g5_hermiticity(dims=(4, 2, 2, 4), seed=2, kappa=0.12):
    """gamma_5 D gamma_5 = D^dagger at mu = 0: <phi, D psi> = <g5 D g5 phi, psi>."""
    cfg = latgen.small_config(dims, seed=seed, nrhs=2)
    U = cfg["U"]
    phi, psi = cfg["b"][0], cfg["b"][1]
    g5 = lambda f: f @ GAMMA5.T
    lhs = np.vdot(phi, W.apply_D(U, kappa, 0.0, psi))
    rhs = np.vdot(g5(W.apply_D(U, kappa, 0.0, g5(phi))), psi)
    return abs(lhs - rhs) / abs(lhs)


def pin_adjoint(dims=(4, 2, 2, 4), seed=3, kappa=0.12, mu=0.05):
    """<phi, D psi> = <D^dagger phi, psi> with the oracle's D^dagger."""
    cfg = latgen.small_config(dims, seed=seed, nrhs=2)
    U = cfg["U"]
    phi, psi = cfg["b"][0], cfg["b"][1]
    lhs = np.vdot(phi, W.apply_D(U, kappa, mu, psi))
    rhs = np.vdot(W.apply_Ddag(U, kappa, mu, phi), psi)
    return abs(lhs - rhs) / abs(lhs)


def pin_translation(dims=(4, 2, 2, 4), seed=4):
    """Shifting links and field by one site in x commutes with H and swaps the parities
    of the even/odd blocks; a shift by two sites keeps them."""
    cfg = latgen.small_config(dims, seed=seed)
    U, psi = cfg["U"], cfg["b"][0]
    err = 0.0
    for a, flip in ((1, 1), (2, 0)):
        sh = lambda f: np.roll(f, a, axis=3)
        for p in (0, 1):
            lhs = W.hop_eo(sh(U), sh(psi), p)
            rhs = sh(W.hop_eo(U, psi, p ^ flip))
            err = max(err, np.abs(lhs - rhs).max())
    return err


ALL_PINS = {
    "free_field": (pin_free_field, 1e-12),
    "u1_background": (lambda: pin_free_field(theta=(0.3, -0.7, 1.1, 0.2)), 1e-12),
    "free_field_L2": (lambda: pin_free_field(dims=(2, 2, 2, 2)), 1e-12),
    "covariance": (pin_covariance, 1e-12),
    "g5_hermiticity": (pin_g5_hermiticity, 1e-13),
    "adjoint": (pin_adjoint, 1e-13),
    "translation": (pin_translation, 1e-13),
}
