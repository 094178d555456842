"""Outer Krylov solver (Sec. 5 uses GMRES around the whole 3D system).

Test infrastructure only (see ``oracle/__init__.py``).

The paper does not say how GMRES is preconditioned or orthogonalised.  This is the
right-preconditioned *flexible* GMRES of Saad (SIAM J. Sci. Comput. 14, 1993): the
preconditioned directions z_j = M^{-1} v_j are stored and the update is x = x0 + Z y, so the
residual estimate stays exact even if M^{-1} is applied in lower precision.  Modified
Gram-Schmidt, complex Givens rotations, x0 = 0 unless given, relative to ||f||_2, and a
true-residual check before returning.

Pinned by solving small systems to 1e-12 against scipy's sparse direct solve
(tests/test_oracle_krylov.py).
"""
import numpy as np
from scipy.linalg import solve_triangular


def _givens(a, b):
    """(c, s, rho): [[c, s], [-conj(s), c]] @ [a, b] = [rho, 0] with c real."""
    if b == 0:
        return 1.0, 0.0j, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b)
    r = np.hypot(abs(a), abs(b))
    c = abs(a) / r
    s = (a / abs(a)) * np.conj(b) / r
    return c, s, (a / abs(a)) * r


def fgmres(matvec, precond, f, tol=1e-6, restart=50, maxit=1000, x0=None):
    """Solve A x = f for one right-hand side.

    Returns (x, iterations, history) where history holds the residual estimate relative to
    ||f|| after every iteration (plus the true one at each restart).
    """
    f = np.asarray(f, np.complex128).ravel()
    nf = np.linalg.norm(f)
    x = np.zeros_like(f) if x0 is None else np.asarray(x0, np.complex128).ravel().copy()
    its = 0
    hist = []
    if nf == 0:
        return x, 0, hist
    while True:
        r = f - matvec(x)
        beta = np.linalg.norm(r)
        hist.append(beta / nf)
        if beta <= tol * nf or its >= maxit:
            return x, its, hist
        m = restart
        V = [r / beta]
        Z = []
        H = np.zeros((m + 1, m), np.complex128)
        cs = np.zeros(m)
        sn = np.zeros(m, np.complex128)
        g = np.zeros(m + 1, np.complex128)
        g[0] = beta
        k = 0
        for j in range(m):
            Z.append(np.asarray(precond(V[j]), np.complex128).ravel())
            w = np.asarray(matvec(Z[j]), np.complex128).ravel()
            its += 1
            for i in range(j + 1):                      # modified Gram-Schmidt
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            V.append(w / H[j + 1, j] if H[j + 1, j] != 0 else w)
            for i in range(j):                          # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j], H[j, j] = _givens(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            hist.append(abs(g[j + 1]) / nf)
            if abs(g[j + 1]) <= tol * nf or its >= maxit:
                break
        y = solve_triangular(H[:k, :k], g[:k])
        for i in range(k):
            x = x + y[i] * Z[i]
