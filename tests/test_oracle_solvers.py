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


def test_fcg_identity_is_cgnr(c0):
    """FCG with the identity on D^dag D x = D^dag b takes CGNR's iterates."""
    cfg, xd = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    D = lambda v: W.apply_D(U, k, 0.0, v)
    Dd = lambda v: W.apply_Ddag(U, k, 0.0, v)
    for n in (1, 4, 10):
        xf, itf, _ = S.fcg(lambda v: Dd(D(v)), Dd(b), lambda r: r, maxiter=n)
        xc, itc, _ = S.cgnr(D, Dd, b, 0.0, maxiter=n)
        assert itf == itc == n
        assert _rel(xf, xc) < 1e-11, n


def test_fcg_normal_with_network_c0(c0):
    """FCG on the normal equations with N N^dag (N: the Neumann-2 network) reaches
    the direct solution, in fewer steps than with the identity."""
    cfg, xd = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    w = ptc.neumann2_weights(k)
    N = lambda v: ptc.network(U, w, v)
    Nd = lambda v: ptc.network_adjoint(U, w, v)
    x, info = S.solve_fcg_normal(U, k, 0.0, b, N, Nd, tol=1e-10)
    assert info["true_rel_resid"] <= 1e-10
    assert _rel(x, xd) < 1e-9
    x1, info1 = S.solve_fcg_normal(U, k, 0.0, b, lambda v: v, lambda v: v, tol=1e-10)
    assert info1["true_rel_resid"] <= 1e-10
    assert info["iterations"] < info1["iterations"]


def test_fcg_directions_are_conjugate_with_a_varying_preconditioner(c0):
    """With a preconditioner that changes every step, each new FCG direction is
    still A-conjugate to the last mmax ones (the step that makes FCG flexible),
    and the iteration still converges."""
    cfg, _ = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    A0 = lambda v: W.apply_Ddag(U, k, 0.0, W.apply_D(U, k, 0.0, v))
    ps = []

    def A(v):
        ps.append(v.copy())
        return A0(v)

    rng = np.random.default_rng(3)
    shape = b.shape

    def precond(r):   # a different positive diagonal every call
        return r * rng.uniform(0.5, 2.0, size=shape)

    c = W.apply_Ddag(U, k, 0.0, b)
    for mmax in (1, 3):
        ps.clear()
        x, it, hist = S.fcg(A, c, precond, eps=(1e-10) ** 2 * W.norm2(c), maxiter=400, mmax=mmax)
        assert hist[-1] <= (1e-10) ** 2 * W.norm2(c), (mmax, it)
        Ap = [A0(p) for p in ps]
        nA = [np.sqrt(W.inner(p, q).real) for p, q in zip(ps, Ap)]
        worst = 0.0
        for i in range(1, min(len(ps), 30)):
            for j in range(max(0, i - mmax), i):
                worst = max(worst, abs(W.inner(ps[i], Ap[j])) / (nA[i] * nA[j]))
        assert worst < 1e-10, (mmax, worst)


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
