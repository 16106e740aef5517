"""Iterative solvers in complex128.

* ``cgnr``: the CGNR template of Fig. "CG" (Sec. 2), step by step in the
  paper's order and notation.
* ``solve_eo_cgnr``: the goal statement ``xx = Dirac^{-1} bb`` with the template
  chain "CGNR schur" (Sec. 2): Schur complement on the odd sites, CGNR on the
  Schur system, reconstruction of the even sites.
* ``bicgstab``: van der Vorst's BiCGStab (SIAM J. Sci. Stat. Comput. 13, 1992),
  an addition to the paper's solvers, on the same Schur system.
* ``fgmres``: flexible GMRES(m) with a right preconditioner that may change
  between iterations (Saad, SIAM J. Sci. Comput. 14, 1993).
* ``fcg``: flexible conjugate gradients (Notay, SIAM J. Sci. Comput. 22,
  2000) for a Hermitian positive definite operator with a preconditioner that
  may vary between steps; ``solve_fcg_normal`` runs it on the normal equations
  D^dag D x = D^dag b with the preconditioner N N^dag of a network N ~ D^-1.
* ``crnr``: the conjugate residual method (Saad, Iterative Methods for Sparse
  Linear Systems, 2nd ed., Alg. 6.20) on the normal equations A^dag A x =
  A^dag b, a residual-minimising counterpart of CGNR (Sec. 5 compares CGNR with
  conjugate-residual variants it does not define).

Stopping rule.  The paper's loop runs while (r|r) > epsilon.  Here epsilon is
(tol * ||b||)^2 with b the full-lattice source, so that the loop stops when
the Schur residual norm is at most tol * ||b||; after reconstruction of the even
sites this residual equals the full-system residual ||b - D x||.
"""
import numpy as np

from . import wilson as W


def cgnr(apply_A, apply_Adag, b, eps, maxiter=100000, x0=None):
    """CGNR for A x = b (Fig. "CG"); x starts at 0 (or at x0, which solves for
    the correction).  Returns (x, iterations, history of n_r)."""
    if x0 is None:
        r = b.copy()
        x = np.zeros_like(b)
    else:
        r = b - apply_A(x0)
        x = x0.copy()
    z = apply_Adag(r)
    p = z.copy()
    n_z = W.norm2(z)
    n_r = W.norm2(r)
    hist = [n_r]
    it = 0
    while n_r > eps and it < maxiter:
        Ap = apply_A(p)
        alpha = n_z / W.norm2(Ap)
        x = x + alpha * p
        r = r - alpha * Ap
        z = apply_Adag(r)
        n_z1 = W.norm2(z)
        beta = n_z1 / n_z
        p = z + beta * p
        n_z = n_z1
        n_r = W.norm2(r)
        hist.append(n_r)
        it += 1
    return x, it, hist


def true_rel_residual(U, kappa, mu, x, b):
    """||b - D x|| / ||b|| over the whole lattice."""
    return np.sqrt(W.norm2(b - W.apply_D(U, kappa, mu, x)) / W.norm2(b))


def solve_eo_cgnr(U, kappa, mu, b, tol=1e-10, maxiter=100000, max_restarts=5):
    """x = D^{-1} b by Schur complement + CGNR.  If the reconstructed solution's
    true residual exceeds tol, CGNR restarts from the current odd solution.
    Returns (x, info) with info = dict(iterations, restarts, true_rel_resid)."""
    bnorm = np.sqrt(W.norm2(b))
    eps = (tol * bnorm) ** 2
    bhat = W.schur_source(U, kappa, mu, b)
    A = lambda v: W.schur(U, kappa, mu, v)
    Ad = lambda v: W.schur(U, kappa, mu, v, dagger=True)
    xo, its, hist = cgnr(A, Ad, bhat, eps, maxiter)
    restarts = 0
    while True:
        x = W.reconstruct_even(U, kappa, mu, b, xo) + xo
        res = true_rel_residual(U, kappa, mu, x, b)
        if res <= tol or restarts >= max_restarts:
            break
        xo, more, _ = cgnr(A, Ad, bhat, eps, maxiter, x0=xo)
        its += more
        restarts += 1
    return x, dict(iterations=its, restarts=restarts, true_rel_resid=res, history=hist)


def crnr(apply_A, apply_Adag, b, eps, maxiter=100000, x0=None):
    """Conjugate residual for the Hermitian system M x = A^dag b, M = A^dag A:
    z is its residual, p the search direction, q = M p, and M-conjugacy of the
    residuals replaces the A-conjugacy of CG.  The residual r = b - A x of the
    original system and u = A p are carried along so that the loop stops on
    (r|r) <= eps, as cgnr does.  Returns (x, iterations, history of n_r)."""
    if x0 is None:
        r = b.copy()
        x = np.zeros_like(b)
    else:
        r = b - apply_A(x0)
        x = x0.copy()
    z = apply_Adag(r)
    v = apply_A(z)
    w = apply_Adag(v)          # M z
    p, q, u = z.copy(), w.copy(), v.copy()
    n_zw = W.inner(z, w).real  # (z | M z), real for Hermitian M
    n_r = W.norm2(r)
    hist = [n_r]
    it = 0
    while n_r > eps and it < maxiter:
        alpha = n_zw / W.norm2(q)
        x = x + alpha * p
        r = r - alpha * u
        z = z - alpha * q
        v = apply_A(z)
        w = apply_Adag(v)
        n_zw1 = W.inner(z, w).real
        beta = n_zw1 / n_zw
        p = z + beta * p
        q = w + beta * q
        u = v + beta * u
        n_zw = n_zw1
        n_r = W.norm2(r)
        hist.append(n_r)
        it += 1
    return x, it, hist


def solve_eo_crnr(U, kappa, mu, b, tol=1e-10, maxiter=100000, max_restarts=5):
    """As solve_eo_cgnr with the conjugate residual method on the Schur system."""
    bnorm = np.sqrt(W.norm2(b))
    eps = (tol * bnorm) ** 2
    bhat = W.schur_source(U, kappa, mu, b)
    A = lambda v: W.schur(U, kappa, mu, v)
    Ad = lambda v: W.schur(U, kappa, mu, v, dagger=True)
    xo, its, hist = crnr(A, Ad, bhat, eps, maxiter)
    restarts = 0
    while True:
        x = W.reconstruct_even(U, kappa, mu, b, xo) + xo
        res = true_rel_residual(U, kappa, mu, x, b)
        if res <= tol or restarts >= max_restarts:
            break
        xo, more, _ = crnr(A, Ad, bhat, eps, maxiter, x0=xo)
        its += more
        restarts += 1
    return x, dict(iterations=its, restarts=restarts, true_rel_resid=res, history=hist)


def bicgstab(apply_A, b, eps, maxiter=100000, x0=None):
    """BiCGStab for A x = b with shadow residual r~ = r_0; stops when (r|r) <= eps.
    On a breakdown (rho or omega = 0) it restarts from the current x."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    it = 0
    while W.norm2(r) > eps and it < maxiter:
        rt = r.copy()
        rho = alpha = omega = 1.0 + 0j
        v = np.zeros_like(b)
        p = np.zeros_like(b)
        while it < maxiter:
            rho1 = W.inner(rt, r)
            if rho1 == 0:
                break
            beta = (rho1 / rho) * (alpha / omega)
            p = r + beta * (p - omega * v)
            v = apply_A(p)
            alpha = rho1 / W.inner(rt, v)
            s = r - alpha * v
            t = apply_A(s)
            tt = W.norm2(t)
            omega = W.inner(t, s) / tt if tt > 0 else 0.0
            x = x + alpha * p + omega * s
            r = s - omega * t
            rho = rho1
            it += 1
            if W.norm2(r) <= eps or omega == 0:
                break
        if omega == 0 or rho1 == 0:
            r = b - apply_A(x)
    return x, it


def solve_eo_bicgstab(U, kappa, mu, b, tol=1e-10, maxiter=100000, max_restarts=5):
    bnorm = np.sqrt(W.norm2(b))
    eps = (tol * bnorm) ** 2
    bhat = W.schur_source(U, kappa, mu, b)
    A = lambda v: W.schur(U, kappa, mu, v)
    xo, its = bicgstab(A, bhat, eps, maxiter)
    restarts = 0
    while True:
        x = W.reconstruct_even(U, kappa, mu, b, xo) + xo
        res = true_rel_residual(U, kappa, mu, x, b)
        if res <= tol or restarts >= max_restarts:
            break
        xo, more = bicgstab(A, bhat, eps, maxiter, x0=xo)
        its += more
        restarts += 1
    return x, dict(iterations=its, restarts=restarts, true_rel_resid=res)


def fgmres(apply_A, b, precond, m=20, tol=1e-10, maxiter=1000, x0=None):
    """Right-preconditioned flexible GMRES(m): x = x0 + Z y, z_j = precond(v_j),
    modified Gram-Schmidt Arnoldi, Givens rotations, restart every m steps.
    Stops when ||b - A x|| <= tol ||b||.  Returns (x, total inner steps, restarts)."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.sqrt(W.norm2(b))
    steps = 0
    cycles = 0
    while steps < maxiter:
        r = b - apply_A(x)
        beta = np.sqrt(W.norm2(r))
        if beta <= tol * bnorm:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m, dtype=np.complex128)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = apply_A(z)
            for i in range(j + 1):
                H[i, j] = W.inner(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.sqrt(W.norm2(w))
            if H[j + 1, j] != 0:
                V.append(w / H[j + 1, j])
            else:
                V.append(np.zeros_like(w))
            for i in range(j):
                hi = H[i, j]
                H[i, j] = np.conj(cs[i]) * hi + np.conj(sn[i]) * H[i + 1, j]
                H[i + 1, j] = -sn[i] * hi + cs[i] * H[i + 1, j]
            a, c = H[j, j], H[j + 1, j]
            den = np.sqrt(abs(a) ** 2 + abs(c) ** 2)
            cs[j], sn[j] = a / den, c / den
            H[j, j] = den
            H[j + 1, j] = 0
            g[j + 1] = -sn[j] * g[j]
            g[j] = np.conj(cs[j]) * g[j]
            k = j + 1
            steps += 1
            if abs(g[j + 1]) <= tol * bnorm or steps >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        for j in range(k):
            x = x + y[j] * Z[j]
        cycles += 1
    return x, steps, cycles


def fcg(apply_A, b, precond, eps=0.0, maxiter=1000, x0=None, mmax=1, done=None):
    """Truncated flexible CG for A x = b, A Hermitian positive definite.  Each
    step preconditions the residual, z = precond(r), makes it A-conjugate to
    the last mmax directions, p = z - sum_i ((A p_i | z) / (p_i | A p_i)) p_i,
    and moves along p by alpha = (p | r) / (p | A p).  With a fixed Hermitian
    positive definite preconditioner (and mmax >= 1) this is preconditioned
    CG; with the identity it is CG.  Stops when (r | r) <= eps, or when
    done(x) is true if given.  Returns (x, iterations, history of (r | r))."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply_A(x) if x0 is not None else b.copy()
    dirs = []   # (p_i, A p_i, (p_i | A p_i)) of the last mmax steps
    hist = [W.norm2(r)]
    it = 0
    while it < maxiter and not (done(x) if done is not None else hist[-1] <= eps):
        z = precond(r)
        p = z.copy()
        for pi, qi, di in dirs:
            p = p - (W.inner(qi, z) / di) * pi
        q = apply_A(p)
        d = W.inner(p, q).real
        if not d > 0:
            break
        alpha = W.inner(p, r) / d
        x = x + alpha * p
        r = r - alpha * q
        dirs.append((p, q, d))
        dirs = dirs[-mmax:]
        hist.append(W.norm2(r))
        it += 1
    return x, it, hist


def solve_fcg_normal(U, kappa, mu, b, apply_N, apply_Ndag, tol=1e-10, maxiter=1000):
    """FCG(1) on D^dag D x = D^dag b, preconditioned by N N^dag, stopping when
    the full-system residual ||b - D x|| is at most tol ||b||."""
    A = lambda v: W.apply_Ddag(U, kappa, mu, W.apply_D(U, kappa, mu, v))
    c = W.apply_Ddag(U, kappa, mu, b)
    lim = tol * np.sqrt(W.norm2(b))
    done = lambda x: np.sqrt(W.norm2(b - W.apply_D(U, kappa, mu, x))) <= lim
    x, it, _ = fcg(A, c, lambda r: apply_N(apply_Ndag(r)), maxiter=maxiter, done=done)
    return x, dict(iterations=it, true_rel_resid=true_rel_residual(U, kappa, mu, x, b))
