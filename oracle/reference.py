"""Test devices that pin the recursive sweep (not part of the method's hot path).

Test infrastructure only (see ``oracle/__init__.py``).

* ``nonrecursive_apply`` -- Algorithm 2 (Sec. 3) along x3 or x2, with every auxiliary problem
  solved exactly by a sparse direct solve.  When the other axis has a single group, the
  recursive Algorithm 6 must reproduce it exactly, since then every quasi-1D "line" is the
  whole auxiliary problem and its block LDU solve is exact.
* ``exact_layer_T`` -- the dense block LDU of Sec. 3 (S_1 = A_11, S_m = A_mm -
  A_{m,m-1} T_{m-1} A_{m-1,m}); T_m = S_m^{-1} is the half-space Green's function restricted
  to layer m, which the moving-PML auxiliary problem approximates.
"""
import numpy as np
import scipy.sparse.linalg as spla

from .problem import axis_profile, assemble_box, helmholtz_matrix
from .partition import groups, window


def nonrecursive_apply(prob, f, axis, first=None):
    """Algorithm 2 with exact auxiliary solves, sweeping along x3 (axis='z') or x2 ('y')."""
    n = prob.n
    first = prob.b if first is None else first
    G = groups(n, first, prob.d)
    A = helmholtz_matrix(prob)
    ax = prob.boundary_axis()
    idx = np.arange(n ** 3).reshape(n, n, n)
    sel = (lambda a, e: idx[a - 1:e].ravel()) if axis == "z" else (lambda a, e: idx[:, a - 1:e, :].ravel())
    blocks = [sel(a, e) for (a, e) in G]
    solvers = []
    for g in range(len(G)):
        w0, w1, fp = window(G, g, prob.p)
        pw = axis_profile(w0, w1, n, prob.b, prob.C, prob.omega, fp, prob.p)
        if axis == "z":
            H = assemble_box(prob.kappa[w0 - 1:w1], ax, ax, pw, prob.h)
            widx = np.arange(H.shape[0]).reshape(w1 - w0 + 1, n, n)
            phys = widx[G[g][0] - w0:].ravel()
        else:
            H = assemble_box(prob.kappa[:, w0 - 1:w1, :], ax, pw, ax, prob.h)
            widx = np.arange(H.shape[0]).reshape(n, w1 - w0 + 1, n)
            phys = widx[:, G[g][0] - w0:, :].ravel()
        solvers.append((spla.splu(H.tocsc()), H.shape[0], phys))

    def T(g, alpha):
        lu, N, phys = solvers[g]
        r = np.zeros((N, alpha.shape[1]), np.complex128)
        r[phys] = alpha
        return lu.solve(r)[phys]

    f = np.asarray(f).reshape(n ** 3, -1)
    u = np.zeros(f.shape, np.complex128)
    for g in range(len(G)):
        rhs = f[blocks[g]].astype(np.complex128)
        if g > 0:
            rhs = rhs - A[blocks[g]][:, blocks[g - 1]] @ u[blocks[g - 1]]
        u[blocks[g]] = T(g, rhs)
    for g in range(len(G) - 2, -1, -1):
        u[blocks[g]] = u[blocks[g]] - T(g, A[blocks[g]][:, blocks[g + 1]] @ u[blocks[g + 1]])
    return u


def exact_layer_T(prob):
    """Dense T_m = S_m^{-1}, m = 1..n, of the layer-by-layer block LDU along x3 (Sec. 3)."""
    n = prob.n
    A = helmholtz_matrix(prob)
    idx = np.arange(n ** 3).reshape(n, n, n)
    L = [idx[m].ravel() for m in range(n)]
    T = []
    for m in range(n):
        S = A[L[m]][:, L[m]].toarray()
        if m > 0:
            S = S - A[L[m]][:, L[m - 1]].toarray() @ T[m - 1] @ A[L[m - 1]][:, L[m]].toarray()
        T.append(np.linalg.inv(S))
    return T
