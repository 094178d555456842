"""Pins of the oracle's 1D nested dissection of the line problems (the parallel alternative
to the block LDU that Sec. 6 proposes): it must return K^{-1} r exactly, as a sparse direct
solve and the block LDU solve of Sec. 3 do, in ceil(log2(n + 1)) dependent levels."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle.nested import NestedDissection
from paper_1502_07266_amd import inputs


def _prob(n, b=3, p=2, d=2, **kw):
    case = inputs.small_case(n=n, b=b, p=p, d=d)
    return O.Problem(n=n, c=case["c"], omega=case["omega"], b=b, C=case["C"], p=p, d=d, **kw)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _lines(prob):
    M = O.RecursiveSweep(prob)
    Gz, Gy = M.Gz, M.Gy
    picks = [(0, 0), (len(Gz) // 2, len(Gy) // 2), (len(Gz) - 1, len(Gy) - 1)]
    return [O.LineFactors(prob, Gz, g, Gy, l) for g, l in picks]


@pytest.mark.parametrize("n", [7, 8, 11])
@pytest.mark.parametrize("fronts", [1, 2])
def test_nested_dissection_equals_direct_and_block_ldu(n, fronts):
    prob = _prob(n, fronts=fronts, fronts_inner=fronts)
    rng = np.random.default_rng(n + 10 * fronts)
    for lf in _lines(prob):
        nd = NestedDissection(lf)
        N = lf.K.shape[0]
        r = rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))
        x_nd = nd.solve(r)
        x_dir = spla.spsolve(lf.K.tocsc(), r)
        assert _rel(x_nd, x_dir) < 1e-10
        assert _rel(x_nd, lf.solve(r)) < 1e-10
        # residual of the system itself (independent of both other solvers)
        assert _rel(lf.K @ x_nd, r) < 1e-10
        assert nd.levels == NestedDissection.expected_levels(n)


@pytest.mark.parametrize("n", [7, 10])
def test_nested_dissection_adjoint(n):
    prob = _prob(n)
    rng = np.random.default_rng(3 * n)
    for lf in _lines(prob):
        nd = NestedDissection(lf)
        N = lf.K.shape[0]
        r = rng.standard_normal(N) + 1j * rng.standard_normal(N)
        x = nd.solve(r, adjoint=True)
        assert _rel(lf.K.conj().T @ x, r) < 1e-10
        assert _rel(x, np.ravel(lf.solve_adjoint(r))) < 1e-10


@pytest.mark.parametrize("n,levels", [(1, 1), (2, 2), (3, 2), (4, 3), (7, 3), (8, 4), (127, 7), (255, 8)])
def test_level_count(n, levels):
    assert NestedDissection.expected_levels(n) == levels
