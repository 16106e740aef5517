"""The oracle's operator against the pins of ``oracle_pins`` (closed forms and
invariants), its even/odd blocks and Schur complement against the block
algebra of the "schur" template, dense brute force on tiny lattices, and a
planted-mistake check that each plausible slip in the hop fails some pin."""
import numpy as np
import pytest

import latgen
from oracle import wilson as W
from oracle import dense
from oracle.gamma import GAMMA5, P_MINUS, P_PLUS

import oracle_pins as pins


@pytest.mark.parametrize("name", list(pins.ALL_PINS))
def test_pin(name):
    fn, tol = pins.ALL_PINS[name]
    assert fn() <= tol


def test_kronecker_layout():
    """(M1 (x) M2) vec(V) = vec(M1 V M2^T) for the 3x4 colour-by-spin block, with the
    canonical flattening k = 4 colour + spin (Sec. 4.2)."""
    rng = np.random.default_rng(0)
    u = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    V = rng.standard_normal((3, 4)) + 1j * rng.standard_normal((3, 4))
    for P in list(P_MINUS) + list(P_PLUS):
        lhs = np.kron(u, P) @ V.reshape(12)
        rhs = W.spin_mul(P, W.colour_mul(u, V)).reshape(12)
        assert np.abs(lhs - rhs).max() < 1e-14


def test_dense_g5_hermiticity_2x4():
    cfg = latgen.small_config((2, 2, 2, 2), seed=5)
    U, k = cfg["U"], 0.12
    D = dense.assemble(lambda f: W.apply_D(U, k, 0.0, f), (2, 2, 2, 2))
    g5 = np.kron(np.eye(16 * 3), GAMMA5)
    assert np.abs(g5 @ D @ g5 - np.conj(D.T)).max() < 1e-15
    Dd = dense.assemble(lambda f: W.apply_Ddag(U, k, 0.3, f), (2, 2, 2, 2))
    D3 = dense.assemble(lambda f: W.apply_D(U, k, 0.3, f), (2, 2, 2, 2))
    assert np.abs(Dd - np.conj(D3.T)).max() < 1e-15


def test_dense_free_spectrum():
    """Eigenvalues of D at U = 1 on 2x2x2x4: 1 - 2k sum cos p +- i sqrt(4k^2 sum sin^2 p + 4k^2 mu^2),
    each 6-fold (3 colours x 2 spin states)."""
    dims, k, mu = (2, 2, 2, 4), 0.11, 0.05
    U = latgen.gauge_field(0, 0, dims, "unit")
    D = dense.assemble(lambda f: W.apply_D(U, k, mu, f), dims)
    ev = np.sort_complex(np.round(np.linalg.eigvals(D), 10))
    want = []
    for n in np.ndindex(*dims):
        p = [2 * np.pi * n[d] / dims[d] for d in range(4)]
        re = 1 - 2 * k * sum(np.cos(p))
        im = np.sqrt(4 * k * k * sum(np.sin(q) ** 2 for q in p) + 4 * k * k * mu * mu)
        want += [re + 1j * im] * 6 + [re - 1j * im] * 6
    want = np.sort_complex(np.round(np.array(want), 10))
    assert np.abs(ev - want).max() < 1e-9


def test_hop_site_matches_hop():
    cfg = latgen.small_config((4, 2, 6, 4), seed=6)
    U, psi = cfg["U"], cfg["b"][0]
    for dag in (False, True):
        full = W.hop(U, psi, dag)
        for site in [(0, 0, 0, 0), (3, 1, 5, 3), (2, 0, 3, 1)]:
            x, y, z, t = site
            assert np.abs(W.hop_site(U, psi, site, dag) - full[t, z, y, x]).max() < 1e-14


def test_eo_blocks():
    """D_ee = D_oo = 1 at mu = 0, and H only couples opposite parities."""
    cfg = latgen.small_config((4, 4, 2, 2), seed=7)
    U, psi = cfg["U"], cfg["b"][0]
    for p in (0, 1):
        pe = W.project(psi, p)
        Dp = W.apply_D(U, 0.12, 0.0, pe)
        assert np.abs(W.project(Dp, p) - pe).max() < 1e-15
        assert np.abs(W.project(W.hop(U, pe), p)).max() == 0


def test_schur_blocks():
    """The Schur operator, source and reconstruction satisfy the block algebra:
    for any x_o, b - D x = b_hat - S x_o on the odd sites and 0 on the even ones,
    where x = (reconstructed x_e, x_o)."""
    cfg = latgen.small_config((4, 2, 2, 4), seed=8, nrhs=2)
    U, b = cfg["U"], cfg["b"][0]
    xo = W.project(cfg["b"][1], 1)
    for mu in (0.0, 0.09):
        k = 0.12
        x = W.reconstruct_even(U, k, mu, b, xo) + xo
        res = b - W.apply_D(U, k, mu, x)
        assert np.abs(W.project(res, 0)).max() < 1e-14
        sres = W.schur_source(U, k, mu, b) - W.schur(U, k, mu, xo)
        assert np.abs(W.project(res, 1) - sres).max() < 1e-14
        # S^dagger is the adjoint of S on odd fields
        phi = W.project(cfg["b"][0], 1)
        lhs = np.vdot(phi, W.schur(U, k, mu, xo))
        rhs = np.vdot(W.schur(U, k, mu, phi, dagger=True), xo)
        assert abs(lhs - rhs) < 1e-13 * abs(lhs)


def test_schur_g5_hermitian():
    cfg = latgen.small_config((4, 2, 2, 4), seed=9)
    U = cfg["U"]
    xo = W.project(cfg["b"][0], 1)
    g5 = lambda f: f @ GAMMA5.T
    a = g5(W.schur(U, 0.12, 0.0, g5(xo)))
    b = W.schur(U, 0.12, 0.0, xo, dagger=True)
    assert np.abs(a - b).max() < 1e-15


# --- planted mistakes ---------------------------------------------------------

def _mutant_hop(kind):
    def hop(U, psi, dagger=False):
        out = np.zeros_like(psi)
        for mu in range(3 if kind == "drop_t" else 4):
            pf, pb = (P_PLUS[mu], P_MINUS[mu]) if dagger else (P_MINUS[mu], P_PLUS[mu])
            if kind == "fwd_sign":
                pf = P_PLUS[mu] if not dagger else P_MINUS[mu]
            u = U[..., mu, :, :]
            if kind == "transpose_link":
                u = np.swapaxes(u, -1, -2)
            ub = W.dagger3(W.shift_bwd(u, mu))
            if kind == "no_dagger":
                ub = W.shift_bwd(u, mu)
            if kind == "bwd_link_here":
                ub = W.dagger3(u)
            spin = (lambda P, f: f @ P) if kind == "spin_untransposed" else W.spin_mul
            fwd, bwd = W.shift_fwd(psi, mu), W.shift_bwd(psi, mu)
            if kind == "swap_shift":
                fwd, bwd = bwd, fwd
            out += spin(pf, W.colour_mul(u, fwd))
            out += spin(pb, W.colour_mul(ub, bwd))
        return out
    return hop


@pytest.mark.parametrize("kind", ["drop_t", "fwd_sign", "transpose_link", "no_dagger",
                                  "bwd_link_here", "spin_untransposed", "swap_shift"])
def test_planted_mistake_is_caught(kind, monkeypatch):
    assert max(fn() / tol for fn, tol in pins.ALL_PINS.values()) <= 1
    monkeypatch.setattr(W, "hop", _mutant_hop(kind))
    worst = max(fn() / tol for fn, tol in pins.ALL_PINS.values())
    assert worst > 1e3, kind
