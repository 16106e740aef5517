"""Oracle solvers against a library direct solve of the assembled operator (the
special case where the iterative methods must reduce to a textbook routine),
the residual semantics of the stopping rule, and the expected behaviour of the
4^4 Haar workload."""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import latgen
from oracle import wilson as W
from oracle import solvers as S
from oracle import dense
from oracle import ptc


@pytest.fixture(scope="module")
def c0():
    cfg = latgen.make_config(0)
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    D = scipy.sparse.csc_matrix(dense.assemble(lambda f: W.apply_D(U, k, 0.0, f), cfg["dims"]))
    x_direct = scipy.sparse.linalg.spsolve(D, b.reshape(-1)).reshape(b.shape)
    return cfg, x_direct


def _rel(a, b):
    return np.sqrt(W.norm2(a - b) / W.norm2(b))


def test_eo_cgnr_c0(c0):
    cfg, xd = c0
    x, info = S.solve_eo_cgnr(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10)
    assert info["true_rel_resid"] <= 1e-10
    # cond(D) ~ 4 here, so the error is at most a few times the residual
    assert _rel(x, xd) < 1e-9
    assert 18 <= info["iterations"] <= 26


def test_eo_bicgstab_c0(c0):
    cfg, xd = c0
    x, info = S.solve_eo_bicgstab(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10)
    assert info["true_rel_resid"] <= 1e-10
    assert _rel(x, xd) < 1e-9


def test_fgmres_c0(c0):
    cfg, xd = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    A = lambda v: W.apply_D(U, k, 0.0, v)
    x, steps, _ = S.fgmres(A, b, lambda v: v, m=20, tol=1e-10)
    assert S.true_rel_residual(U, k, 0.0, x, b) <= 1e-10
    assert _rel(x, xd) < 1e-9
    # a Neumann-series preconditioner (the 2-layer network's closed-form weights)
    w = ptc.neumann2_weights(k)
    xn, stepsn, _ = S.fgmres(A, b, lambda v: ptc.network(U, w, v), m=20, tol=1e-10)
    assert S.true_rel_residual(U, k, 0.0, xn, b) <= 1e-10
    assert stepsn < steps


def test_eo_crnr_c0(c0):
    cfg, xd = c0
    x, info = S.solve_eo_crnr(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10)
    assert info["true_rel_resid"] <= 1e-10
    assert _rel(x, xd) < 1e-9


def test_crnr_minimises_normal_residual_over_krylov_space():
    """Conjugate residual on M = S^dag S: after k steps from x = 0, the normal
    residual z_k = S^dag (b - S x_k) is the smallest over x in the Krylov space
    span{z0, M z0, .., M^(k-1) z0} (checked by a least-squares solve on that
    basis), and ||z_k|| never increases.  CG's iterate minimises a different
    norm and fails the first check."""
    cfg = latgen.small_config((4, 2, 2, 4), seed=12, kind="haar")
    U, k, b = cfg["U"], 0.12, cfg["b"][0]
    bh = W.schur_source(U, k, 0.0, b)
    A = lambda v: W.schur(U, k, 0.0, v)
    Ad = lambda v: W.schur(U, k, 0.0, v, dagger=True)
    M = lambda v: Ad(A(v))
    odd = W.parity_field(W.dims_of(b)) == 1
    flat = lambda f: f[odd].reshape(-1)
    z0 = Ad(bh)
    basis = [z0]
    for _ in range(5):
        basis.append(M(basis[-1]))
    prev = np.inf
    for steps in range(1, 6):
        x, _, _ = S.crnr(A, Ad, bh, 0.0, maxiter=steps)
        zk = np.sqrt(W.norm2(Ad(bh - A(x))))
        K = np.stack([flat(v) for v in basis[:steps]], axis=1)
        MK = np.stack([flat(M(v)) for v in basis[:steps]], axis=1)
        y, *_ = np.linalg.lstsq(MK, flat(z0), rcond=None)
        best = np.linalg.norm(flat(z0) - MK @ y)
        assert zk <= best * (1 + 1e-8) + 1e-12, (steps, zk, best)
        assert zk <= prev * (1 + 1e-12)
        prev = zk
        xcg, _, _ = S.cgnr(A, Ad, bh, 0.0, maxiter=steps)
        if steps >= 2:
            assert np.sqrt(W.norm2(Ad(bh - A(xcg)))) > best * (1 + 1e-6)


def test_twisted_mass_schur():
    cfg = latgen.small_config((4, 2, 2, 4), seed=11)
    U, b = cfg["U"], cfg["b"][0]
    k, mu = 0.12, 0.2
    x, info = S.solve_eo_cgnr(U, k, mu, b, tol=1e-11)
    D = dense.assemble(lambda f: W.apply_D(U, k, mu, f), cfg["dims"])
    xd = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    assert _rel(x, xd) < 1e-10


def test_stopping_rule_is_full_residual():
    """Right after CGNR stops, the Schur residual equals the full residual (the paper's
    stopping quantity (r|r) is the squared full residual norm after reconstruction)."""
    cfg = latgen.small_config((4, 4, 2, 2), seed=12)
    U, b, k = cfg["U"], cfg["b"][0], 0.12
    bhat = W.schur_source(U, k, 0.0, b)
    xo, its, hist = S.cgnr(lambda v: W.schur(U, k, 0.0, v), lambda v: W.schur(U, k, 0.0, v, True),
                           bhat, eps=1e-12 * W.norm2(b), maxiter=6)
    x = W.reconstruct_even(U, k, 0.0, b, xo) + xo
    full = W.norm2(b - W.apply_D(U, k, 0.0, x))
    rec = W.norm2(bhat - W.schur(U, k, 0.0, xo))
    assert abs(full - rec) <= 1e-10 * full
    # the recursively updated residual tracks the true one closely at this stage
    assert abs(hist[-1] - rec) <= 1e-8 * rec


def test_maxiter_not_converged():
    cfg = latgen.make_config(0)
    x, info = S.solve_eo_cgnr(cfg["U"], cfg["kappa"], 0.0, cfg["b"][0], tol=1e-10, maxiter=1, max_restarts=0)
    assert info["iterations"] == 1 and info["true_rel_resid"] > 1e-10
