"""Flexible GMRES(m) with right preconditioning.

Test infrastructure (see the package header).

The outer solver of Sections 2.2 and 5: restarted flexible GMRES (Saad,
SIAM J. Sci. Comput. 1993) with the multigrid cycle as a right
preconditioner that may change from one iteration to the next; zero
initial guess; stop when the relative residual ||b - A x|| / ||b|| reaches
the tolerance; the iteration count is the number of preconditioner
applications.  Arnoldi uses modified Gram-Schmidt; the least-squares
problem is reduced with complex Givens rotations.  Everything in float64.
"""
import numpy as np


def givens(a, b):
    """complex rotation (c real, s complex) with
    [c s; -conj(s) c] [a; b] = [r; 0]."""
    if b == 0:
        return 1.0, 0.0 + 0.0j
    if a == 0:
        return 0.0, np.conj(b) / abs(b)
    den = np.hypot(abs(a), abs(b))
    c = abs(a) / den
    s = (a / abs(a)) * np.conj(b) / den
    return c, s


def fgmres(matvec, b, precond=None, restart=5, tol=1e-6, maxit=500, x0=None,
           history=None):
    """Solve A x = b.  Returns (x, info) with info = dict(iters, relres,
    converged, restarts).  `history`, if a list, receives the estimated
    relative residual after every iteration."""
    b = np.asarray(b)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b, dtype=np.complex128) if x0 is None else np.array(x0, dtype=np.complex128)
    if precond is None:
        precond = lambda v: v
    if nb == 0:
        return x, dict(iters=0, relres=0.0, converged=True, restarts=0)
    r = b - matvec(x)
    beta = np.linalg.norm(r)
    iters, restarts = 0, 0
    m = restart
    while True:
        if beta / nb <= tol or iters >= maxit:
            break
        V = [r / beta]
        Z = []
        Hm = np.zeros((m + 1, m), dtype=np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=np.complex128)
        g = np.zeros(m + 1, dtype=np.complex128)
        g[0] = beta
        jend = -1
        for j in range(m):
            z = precond(V[j])
            Z.append(z)
            w = matvec(z)
            iters += 1
            for i in range(j + 1):
                Hm[i, j] = np.vdot(V[i], w)
                w = w - Hm[i, j] * V[i]
            Hm[j + 1, j] = np.linalg.norm(w)
            if Hm[j + 1, j] != 0:
                V.append(w / Hm[j + 1, j])
            else:
                V.append(np.zeros_like(w))
            for i in range(j):
                t = cs[i] * Hm[i, j] + sn[i] * Hm[i + 1, j]
                Hm[i + 1, j] = -np.conj(sn[i]) * Hm[i, j] + cs[i] * Hm[i + 1, j]
                Hm[i, j] = t
            cs[j], sn[j] = givens(Hm[j, j], Hm[j + 1, j])
            Hm[j, j] = cs[j] * Hm[j, j] + sn[j] * Hm[j + 1, j]
            Hm[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            jend = j
            if history is not None:
                history.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) / nb <= tol or iters >= maxit:
                break
        k = jend + 1
        y = np.zeros(k, dtype=np.complex128)
        for i in range(k - 1, -1, -1):
            y[i] = (g[i] - Hm[i, i + 1:k] @ y[i + 1:k]) / Hm[i, i]
        for i in range(k):
            x = x + y[i] * Z[i]
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        restarts += 1
    return x, dict(iters=iters, relres=beta / nb, converged=beta / nb <= tol,
                   restarts=restarts)
