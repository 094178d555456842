"""Adjoint-state gradient of a receiver misfit (not in the paper; derived from eq. (3)).

Test infrastructure only (see ``oracle/__init__.py``).

J(c) = 1/2 sum_s || P u_s - d_s ||^2 with A(c) u_s = f_s, P the restriction to all nodes of
one x3-layer.  In eq. (3) the velocity enters only through the diagonal term omega^2/c^2
(the stretchings s_d do not depend on c, Sec. 2), so dA/dc_p = -2 omega^2 / c_p^3 e_p e_p^T.
With lambda_s solving A^H lambda_s = P^T (P u_s - d_s):

    dJ/dc_p = (2 omega^2 / c_p^3) * Re sum_s conj(lambda_s,p) u_s,p .

Pinned by central finite differences of J (tests/test_oracle_gradient.py).
"""
import numpy as np
import scipy.sparse.linalg as spla

from .problem import helmholtz_matrix


def misfit_and_gradient(prob, F, plane_k, d_obs, solve=None, solve_adjoint=None):
    """Return (J, grad, U) for sources F (shape (S, n, n, n), [k, j, i] per source).

    plane_k is the 1-based x3 index of the receiver layer; d_obs has shape (S, n, n).
    ``solve(A, F)`` / ``solve_adjoint(AH, G)`` default to a sparse direct solve of eq. (3).
    """
    n = prob.n
    A = helmholtz_matrix(prob).tocsc()
    AH = A.conj().T.tocsc()
    if solve is None:
        lu = spla.splu(A)
        solve = lambda M, B: lu.solve(B)
    if solve_adjoint is None:
        luh = spla.splu(AH)
        solve_adjoint = lambda M, B: luh.solve(B)
    S = F.shape[0]
    Fm = F.reshape(S, -1).T.astype(np.complex128)
    U = np.asarray(solve(A, Fm)).reshape(n, n, n, S)
    res = U[plane_k - 1] - np.moveaxis(np.asarray(d_obs), 0, -1)       # (n, n, S)
    J = 0.5 * float(np.sum(np.abs(res) ** 2))
    G = np.zeros((n, n, n, S), np.complex128)
    G[plane_k - 1] = res                                               # P^T (P u - d)
    Lam = np.asarray(solve_adjoint(AH, G.reshape(-1, S))).reshape(n, n, n, S)
    grad = (2.0 * prob.omega ** 2 / prob.c ** 3) * np.real(np.sum(np.conj(Lam) * U, axis=-1))
    return J, grad, np.moveaxis(U, -1, 0)
