"""Compositions of solver x system x right preconditioner (oracle/compose.py),
pinned by things other than themselves:

* every composition reaches the direct solution (scipy's sparse LU of the
  assembled 4^4 operator) to the error its residual allows;
* with the identity as preconditioner, right-preconditioned BiCGStab takes
  plain BiCGStab's iterates, and FCG on the Schur normal equations takes CGNR's;
* with the exact inverse as preconditioner (a dense solve), BiCGStab and
  FGMRES converge in one step;
* the Schur preconditioner built from the exact D^-1, v -> P_o D^-1 (0 (+) v),
  is the exact S^-1 (the reading of how a full-lattice map preconditions the
  odd-site system);
* the Neumann-2 network as preconditioner cuts the iterations of every
  composition."""
import numpy as np
import pytest
import scipy.sparse
import scipy.sparse.linalg

import latgen
from oracle import compose as C
from oracle import dense, ptc
from oracle import solvers as S
from oracle import wilson as W


@pytest.fixture(scope="module")
def c0():
    cfg = latgen.make_config(0)
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    D = scipy.sparse.csc_matrix(dense.assemble(lambda f: W.apply_D(U, k, 0.0, f), cfg["dims"]))
    lu = scipy.sparse.linalg.splu(D)
    x_direct = lu.solve(b.reshape(-1)).reshape(b.shape)
    Dinv = lambda v: lu.solve(v.reshape(-1)).reshape(v.shape)
    return cfg, x_direct, Dinv


def _rel(a, b):
    return np.sqrt(W.norm2(a - b) / W.norm2(b))


COMBOS = [(s, k) for s in ("fgmres", "bicgstab", "fcg") for k in ("full", "schur")]


@pytest.mark.parametrize("solver,kind", COMBOS)
@pytest.mark.parametrize("with_net", [False, True], ids=["identity", "neumann2"])
def test_compositions_reach_direct_solution(c0, solver, kind, with_net):
    cfg, xd, _ = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    M = Md = None
    if with_net:
        w = ptc.neumann2_weights(k)
        M, Md = (lambda v: ptc.network(U, w, v)), (lambda v: ptc.network_adjoint(U, w, v))
    x, info = C.solve(U, k, 0.0, b, solver, kind, M, Md, tol=1e-10)
    assert info["true_rel_resid"] <= 1e-10, info
    assert _rel(x, xd) < 1e-9   # cond(D) ~ 4


@pytest.mark.parametrize("solver,kind", COMBOS)
def test_network_cuts_iterations(c0, solver, kind):
    cfg, _, _ = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    w = ptc.neumann2_weights(k)
    _, i0 = C.solve(U, k, 0.0, b, solver, kind, tol=1e-10)
    _, i1 = C.solve(U, k, 0.0, b, solver, kind, lambda v: ptc.network(U, w, v),
                    lambda v: ptc.network_adjoint(U, w, v), tol=1e-10)
    assert i1["iterations"] < i0["iterations"], (i0, i1)


def test_bicgstab_identity_is_plain_bicgstab(c0):
    cfg, _, _ = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    A = lambda v: W.schur(U, k, 0.0, v)
    bh = W.schur_source(U, k, 0.0, b)
    for n in (1, 3, 7):
        xr, itr = C.bicgstab_right(A, bh, lambda v: v.copy(), 0.0, maxiter=n)
        xp, itp = S.bicgstab(A, bh, 0.0, maxiter=n)
        assert itr == itp == n
        assert _rel(xr, xp) < 1e-12, n


def test_fcg_schur_identity_is_cgnr(c0):
    """FCG with the identity on S^dag S x_o = S^dag b_hat takes CGNR's iterates
    on the Schur system (the paper's plain method)."""
    cfg, _, _ = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    A = lambda v: W.schur(U, k, 0.0, v)
    Ad = lambda v: W.schur(U, k, 0.0, v, dagger=True)
    bh = W.schur_source(U, k, 0.0, b)
    for n in (1, 5, 12):
        xf, itf, _ = S.fcg(lambda v: Ad(A(v)), Ad(bh), lambda r: r, maxiter=n)
        xc, itc, _ = S.cgnr(A, Ad, bh, 0.0, maxiter=n)
        assert itf == itc == n
        assert _rel(xf, xc) < 1e-11, n


def test_exact_inverse_preconditioner_converges_in_one_step(c0):
    cfg, xd, Dinv = c0
    U, k, b = cfg["U"], cfg["kappa"], cfg["b"][0]
    A = lambda v: W.apply_D(U, k, 0.0, v)
    x, it = C.bicgstab_right(A, b, Dinv, (1e-12 * np.sqrt(W.norm2(b))) ** 2, maxiter=5)
    assert it == 1 and _rel(x, xd) < 1e-12
    x, steps, _ = S.fgmres(A, b, Dinv, m=20, tol=1e-12)
    assert steps == 1 and _rel(x, xd) < 1e-12


def test_schur_preconditioner_of_exact_inverse_is_schur_inverse(c0):
    cfg, _, Dinv = c0
    U, k = cfg["U"], cfg["kappa"]
    v = W.project(latgen.gaussian_source(0, 5, cfg["dims"], 1)[0], 1)
    MS = C.schur_precond(Dinv)
    y = MS(v)
    assert np.count_nonzero(W.project(y, 0)) == 0
    # S (M_S v) = v on the odd sites
    assert _rel(W.project(W.schur(U, k, 0.0, y), 1), v) < 1e-12
    # and with a twisted mass
    mu = 0.3
    D = scipy.sparse.csc_matrix(dense.assemble(lambda f: W.apply_D(U, k, mu, f), cfg["dims"]))
    lu = scipy.sparse.linalg.splu(D)
    MS = C.schur_precond(lambda u: lu.solve(u.reshape(-1)).reshape(u.shape))
    assert _rel(W.project(W.schur(U, k, mu, MS(v)), 1), v) < 1e-12
