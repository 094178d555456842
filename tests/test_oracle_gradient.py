"""Pin of the oracle's adjoint-state misfit gradient against central finite differences."""
import numpy as np

import oracle as O
from paper_1502_07266_amd import inputs


def test_adjoint_gradient_matches_central_differences():
    n, b = 11, 3
    case = inputs.small_case(n=n, b=b, p=b)
    c = case["c"]
    prob = O.Problem(n=n, c=c, omega=case["omega"], b=b, C=case["C"], p=b)
    nodes = [(5, 6, b + 1), (7, 4, b + 1)]
    F = inputs.sources(n, nodes)
    plane = n - b
    # synthetic data from a smoother medium
    prob0 = O.Problem(n=n, c=np.full((n, n, n), 1.15), omega=prob.omega, b=b, C=prob.C, p=b)
    _, _, U0 = O.misfit_and_gradient(prob0, F, plane, np.zeros((2, n, n)))
    d_obs = U0[:, plane - 1]
    J, grad, _ = O.misfit_and_gradient(prob, F, plane, d_obs)
    assert J > 0
    eps = 1e-4
    for cell in inputs.fd_cells(n, b, 6):
        i, j, k = cell
        cp, cm = c.copy(), c.copy()
        cp[k - 1, j - 1, i - 1] += eps
        cm[k - 1, j - 1, i - 1] -= eps
        Jp = O.misfit_and_gradient(O.Problem(n=n, c=cp, omega=prob.omega, b=b, C=prob.C, p=b), F, plane, d_obs)[0]
        Jm = O.misfit_and_gradient(O.Problem(n=n, c=cm, omega=prob.omega, b=b, C=prob.C, p=b), F, plane, d_obs)[0]
        fd = (Jp - Jm) / (2 * eps)
        g = grad[k - 1, j - 1, i - 1]
        assert abs(fd - g) <= 1e-5 * max(abs(g), 1e-3 * np.max(np.abs(grad))), (cell, fd, g)
