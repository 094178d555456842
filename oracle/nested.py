"""1D nested dissection of a quasi-1D line problem: the alternative to the block LDU that the
paper's closing discussion (Sec. 6) proposes because its halves can be processed in
parallel at essentially the same cost.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The line matrix K of ``LineFactors`` is block tridiagonal in x1: n blocks of B unknowns,
coupled only to their x1-neighbours.  Nested dissection takes the middle block s of an index
range as its separator.  With s removed, the blocks below and above it are two independent
smaller line problems of the same kind; each is solved (the same way, recursively) for its
right-hand side and for the columns that couple it to s.  The separator then follows from its
Schur complement, S = K_ss - K_s,s-1 (K_low^{-1} K_low,s) - K_s,s+1 (K_high^{-1} K_high,s),
and the halves are corrected by their coupling to the separator's value.  It is Gaussian
elimination of K in another order (separators last), so the result is K^{-1} r up to
rounding, and the two halves of every level are independent: a solve has ceil(log2(n + 1))
dependent levels instead of the n steps of the block LDU.

Parity status: pinned (tests/test_oracle_nested.py) against a sparse direct solve of K, the
block LDU solve of ``LineFactors``, and the level count.  The HIP line solver of the same
elimination order (block cyclic reduction, helm_set_line_solver) is checked against the
oracle's line solves and sweeps in tests/test_gpu_nd.py.
"""
import math

import numpy as np


class NestedDissection:
    """Nested-dissection solver of the line problem held by a ``LineFactors`` object."""

    def __init__(self, lf):
        self.n, self.B = lf.n, lf.B
        self.sel = lf.sel
        self.D = [lf.K[s][:, s].toarray() for s in lf.sel]
        self.Kc = {key: m.toarray() for key, m in lf.Kc.items()}
        self.levels = 0

    def _solve(self, lo, hi, F, depth, adjoint):
        """X with K[lo:hi, lo:hi] X = F; F and X are lists of (B x m) arrays, block lo first."""
        if hi <= lo:
            return []
        self.levels = max(self.levels, depth + 1)
        D = (lambda i: self.D[i].conj().T) if adjoint else (lambda i: self.D[i])
        Kc = (lambda i, j: self.Kc[(j, i)].conj().T) if adjoint else (lambda i, j: self.Kc[(i, j)])
        if hi - lo == 1:
            return [np.linalg.solve(D(lo), F[0])]
        s = (lo + hi) // 2
        m = F[0].shape[1]
        B = self.B
        # each half: its right-hand side and, beside it, its coupling columns to the separator
        halves = []
        for a, b, nb in ((lo, s, s - 1), (s + 1, hi, s + 1)):
            if b <= a:
                halves.append(None)
                continue
            E = [np.zeros((B, B), np.complex128) for _ in range(a, b)]
            E[nb - a] = Kc(nb, s)
            G = [np.hstack([F[i - lo], E[i - a]]) for i in range(a, b)]
            XY = self._solve(a, b, G, depth + 1, adjoint)
            halves.append((a, nb, [v[:, :m] for v in XY], [v[:, m:] for v in XY]))
        S = D(s).copy()
        rhs = F[s - lo].copy()
        for h in halves:
            if h is None:
                continue
            a, nb, X, Y = h
            S = S - Kc(s, nb) @ Y[nb - a]
            rhs = rhs - Kc(s, nb) @ X[nb - a]
        xs = np.linalg.solve(S, rhs)
        out = [None] * (hi - lo)
        out[s - lo] = xs
        for h in halves:
            if h is None:
                continue
            a, nb, X, Y = h
            for k in range(len(X)):
                out[a + k - lo] = X[k] - Y[k] @ xs
        return out

    def solve(self, r, adjoint=False):
        """K^{-1} r (or K^{-H} r); r is a vector or a matrix of columns on the line grid."""
        r = np.asarray(r, np.complex128)
        vec = r.ndim == 1
        R = r[:, None] if vec else r
        self.levels = 0
        X = self._solve(0, self.n, [R[s] for s in self.sel], 0, adjoint)
        out = np.zeros(R.shape, np.complex128)
        for i, s in enumerate(self.sel):
            out[s] = X[i]
        return out[:, 0] if vec else out

    @staticmethod
    def expected_levels(n):
        """Dependent levels of a solve: the recursion depth of halving n blocks."""
        return math.ceil(math.log2(n + 1))
