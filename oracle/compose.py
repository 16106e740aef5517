"""Compositions of a Krylov solver, the system it runs on and a right
preconditioner, the runtime counterpart of the right-to-left template chains
of Sec. 2 and Sec. 3.1 ("CGNR schur"): the solver template applied to the
system a transformation template produced.

* System "full": D x = b on the whole lattice.
* System "schur": S x_o = b_hat on the odd sites (template "schur", Fig.
  "schur"), then x_e = A^-1 (b_e + kappa H_eo x_o).
* Preconditioner: a map M ~ A^-1 of the system (for the full system, the
  network N ~ D^-1; for the Schur system, M_S v = P_o N (0 (+) v): the odd part
  of N applied to v placed on the odd sites, since the odd part of D^-1 (0 (+) v)
  is S^-1 v), or the identity.

Solvers: flexible GMRES(m) with M as right preconditioner; BiCGStab with M as
right preconditioner (Barrett et al., Templates for the Solution of Linear
Systems, SIAM 1994, the preconditioned BiCGStab); flexible CG on the normal
equations A^dag A x = A^dag b with M M^dag.  All in complex128; half-fields are
full-lattice arrays that are zero on the other parity (as in wilson.schur).
"""
import numpy as np

from . import solvers, wilson as W


def bicgstab_right(apply_A, b, precond, eps, maxiter=100000, x0=None):
    """BiCGStab for A x = b with the right preconditioner M (precond): the
    directions p and s are preconditioned, p^ = M p and s^ = M s, and x moves
    along them; with M the identity these are plain BiCGStab's iterates.  Stops
    when (r|r) <= eps.  Returns (x, iterations)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    rt = r.copy()
    rho = alpha = omega = 1.0 + 0j
    v = np.zeros_like(b)
    p = np.zeros_like(b)
    it = 0
    while W.norm2(r) > eps and it < maxiter:
        rho1 = W.inner(rt, r)
        if rho1 == 0:
            break
        beta = (rho1 / rho) * (alpha / omega)
        p = r + beta * (p - omega * v)
        ph = precond(p)
        v = apply_A(ph)
        alpha = rho1 / W.inner(rt, v)
        s = r - alpha * v
        sh = precond(s)
        t = apply_A(sh)
        tt = W.norm2(t)
        omega = W.inner(t, s) / tt if tt > 0 else 0.0
        x = x + alpha * ph + omega * sh
        r = s - omega * t
        rho = rho1
        it += 1
        if omega == 0:
            break
    return x, it


def system(U, kappa, mu, b, kind):
    """(apply_A, apply_Adag, rhs) of the system the solver runs on."""
    if kind == "full":
        return (lambda v: W.apply_D(U, kappa, mu, v), lambda v: W.apply_Ddag(U, kappa, mu, v), b)
    if kind == "schur":
        return (lambda v: W.schur(U, kappa, mu, v), lambda v: W.schur(U, kappa, mu, v, dagger=True),
                W.schur_source(U, kappa, mu, b))
    raise ValueError(kind)


def schur_precond(apply_M):
    """M_S v = P_o M (0 (+) v) for a full-lattice map M ~ D^-1."""
    return lambda v: W.project(apply_M(W.project(v, 1)), 1)


def solve(U, kappa, mu, b, solver, kind, apply_M=None, apply_Mdag=None, tol=1e-10, m=20, maxiter=10000):
    """x = D^-1 b by `solver` ("fgmres", "bicgstab", "fcg") on the system `kind`
    ("full" or "schur") with the right preconditioner apply_M (full-lattice map,
    None: the identity; FCG also needs its adjoint apply_Mdag).  Returns (x, info)."""
    A, Adag, rhs = system(U, kappa, mu, b, kind)
    ident = lambda v: v.copy()
    M = ident if apply_M is None else (schur_precond(apply_M) if kind == "schur" else apply_M)
    Md = ident if apply_Mdag is None else (schur_precond(apply_Mdag) if kind == "schur" else apply_Mdag)
    bnorm = np.sqrt(W.norm2(b))
    if solver == "fgmres":
        y, it, _ = solvers.fgmres(A, rhs, M, m=m, tol=tol * bnorm / np.sqrt(W.norm2(rhs)), maxiter=maxiter)
    elif solver == "bicgstab":
        y, it = bicgstab_right(A, rhs, M, (tol * bnorm) ** 2, maxiter)
    elif solver == "fcg":
        c = Adag(rhs)
        lim = tol * bnorm
        done = lambda z: np.sqrt(W.norm2(rhs - A(z))) <= lim
        y, it, _ = solvers.fcg(lambda v: Adag(A(v)), c, lambda r: M(Md(r)), maxiter=maxiter, done=done)
    else:
        raise ValueError(solver)
    x = y if kind == "full" else W.reconstruct_even(U, kappa, mu, b, y) + y
    return x, dict(iterations=it, true_rel_resid=solvers.true_rel_residual(U, kappa, mu, x, b))
