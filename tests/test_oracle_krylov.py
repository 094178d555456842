"""Pins of the oracle's flexible GMRES (the outer solver of Sec. 5) against sparse direct
solves."""
import numpy as np
import scipy.sparse.linalg as spla

import oracle as O
from paper_1502_07266_amd import inputs


def _prob(n=11, b=3, p=3):
    case = inputs.small_case(n=n, b=b, p=p)
    return O.Problem(n=n, c=case["c"], omega=case["omega"], b=b, C=case["C"], p=p)


def test_givens_annihilates():
    from oracle.krylov import _givens
    for a, b in [(1 + 2j, 3.0), (0j, 2.0), (-0.5j, 1e-3), (4.0 + 0j, 0.0)]:
        c, s, rho = _givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, b])
        assert abs(out[1]) < 1e-14 * max(1, abs(a), abs(b))
        assert abs(out[0] - rho) < 1e-14 * max(1, abs(rho))
        assert np.allclose(G.conj().T @ G, np.eye(2), atol=1e-14)


def test_fgmres_with_sweep_matches_direct_solve():
    prob = _prob()
    M = O.RecursiveSweep(prob)
    f = inputs.random_rhs(11, 1, seed=4).reshape(-1)
    x_ref = spla.spsolve(M.A.tocsc(), f)
    x, its, hist = O.fgmres(lambda v: M.A @ v, lambda v: M.apply(v)[:, 0], f, tol=1e-12, restart=50)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-9
    assert its < 40
    assert hist[-1] <= 1e-12


def test_fgmres_restart_and_identity_preconditioner():
    """Restarted, unpreconditioned: still converges (slowly) to the same solution; restart
    length 5 forces several restarts."""
    prob = _prob(n=7, b=2, p=2)
    A = O.helmholtz_matrix(prob)
    f = inputs.random_rhs(7, 1, seed=2).reshape(-1)
    x_ref = spla.spsolve(A.tocsc(), f)
    M = O.RecursiveSweep(prob)
    x, its, hist = O.fgmres(lambda v: A @ v, lambda v: M.apply(v)[:, 0], f, tol=1e-11, restart=5)
    assert np.linalg.norm(x - x_ref) / np.linalg.norm(x_ref) < 1e-8
    assert its > 5
    x2, its2, _ = O.fgmres(lambda v: A @ v, lambda v: v, f, tol=1e-6, restart=400, maxit=400)
    assert np.linalg.norm(A @ x2 - f) / np.linalg.norm(f) <= 1e-6


def test_manufactured_solution():
    prob = _prob()
    M = O.RecursiveSweep(prob)
    u_star = inputs.random_rhs(11, 1, seed=9).reshape(-1)
    f = M.A @ u_star
    x, its, _ = O.fgmres(lambda v: M.A @ v, lambda v: M.apply(v)[:, 0], f, tol=1e-12)
    assert np.linalg.norm(x - u_star) / np.linalg.norm(u_star) < 1e-8
