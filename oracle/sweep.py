"""Sec. 4 of the paper: the recursive sweeping preconditioner.

Test infrastructure only (see ``oracle/__init__.py``).

* ``LineFactors``    -- one quasi-1D auxiliary problem (Sec. 4.1, moving PML next to the
                        y-group, Fig. 3), factored by the block LDU of Sec. 3 with the x1
                        index as block index (x3 and x2 grouped first, x1 last), the blocks
                        eliminated upwards, downwards or from both ends towards the middle.
* ``SlabSweep``      -- one quasi-2D auxiliary problem (H_b or H_m of Sec. 3) and its inner
                        sweep: Algorithm 3 (setup) and Algorithm 4 (apply).
* ``RecursiveSweep`` -- Algorithm 5 (setup) and Algorithm 6 (apply) of Sec. 4.2, with the
                        group/window generalisation of the Sec. 4.2 implementation notes,
                        and the adjoint apply.

Every coupling block (A_{G_g,G_{g-1}}, the slab's tilde-A blocks, the line's off-diagonal
blocks) is sliced out of the assembled sparse matrix, and every Schur update uses the full
block product of Sec. 3 / Sec. 4.1 (S_m = A_mm - A_{m,m-1} T_{m-1} A_{m-1,m}); nothing here
relies on those blocks being multiples of the identity.

Adjoint.  Algorithm 6 computes M^{-1} = U^{-1} D^{-1} L^{-1} for the block factors
L = I + (A_{g,g-1} TT_{g-1}), D = diag(TT_g^{-1}), U = I + (TT_g A_{g,g+1}).  Taking the
conjugate transpose of that product gives M^{-H} = L^{-H} D^{-H} U^{-H}, which is the same
forward-then-backward pass with every coupling block taken from A^H and every TT_g replaced
by TT_g^H; the same holds one level down (Algorithm 4 with the slab matrix) and for the
line solves (K^{-H} = L^{-H} D^{-H} U^{-H} with the block LDU factors).  Pinned by the dot
test <M^{-1}x, y> = <x, M^{-H}y>.

Pins (tests/test_oracle_sweep.py): each line's block LDU reproduces its matrix and its
solve equals a dense solve, in every elimination order; the first block eliminated has
T = K_ii^{-1} and the last one T = (K^{-1})_ii; degenerate partitions reduce Algorithm 6 to an exact solve
(first groups = whole axis) or to the non-recursive Algorithm 2 with exact auxiliary solves
(along x3 or along x2); the moving PML makes the auxiliary restriction approach the exact
Schur-complement inverse T_m of Sec. 3 as p grows; M^{-1} is linear; the dot test above.
"""
import numpy as np
import scipy.sparse as sp

from .problem import axis_profile, assemble_box, helmholtz_matrix
from .partition import groups, groups_two_fronts, window, window_fronts


def _dense_times_sparse(M, S):
    """M @ S for a dense M and a sparse S."""
    return np.asarray((S.T @ M.T).T)


def _cols(v):
    """View a vector as an (N, R) array of right-hand sides."""
    v = np.asarray(v)
    return v.reshape(v.shape[0], -1)


def elimination_order(n, kind="up"):
    """Order in which the x1-blocks 0..n-1 of a line are eliminated by its block LDU.

    "up": 0, 1, ..., n-1 (the order of Sec. 3).  "down": n-1, ..., 0.  "two-sided": blocks
    0..m-1 upwards and n-1..m+1 downwards, the middle block m = n//2 last.  Every order
    eliminates an end block of the remaining chain, so no fill is created and the block LDU
    stays exact; only the factors differ.
    """
    if kind == "up":
        return list(range(n))
    if kind == "down":
        return list(range(n - 1, -1, -1))
    if kind == "two-sided":
        m = n // 2
        return list(range(m)) + list(range(n - 1, m, -1)) + [m]
    raise ValueError(kind)


class LineFactors:
    """Quasi-1D auxiliary problem of (z-group zg, y-group yg) and its block LDU (Sec. 4.1).

    The grid is x1 = 1..n times the y-window times the z-window.  Within the block of x1
    index i the unknowns (jj, kk) are ordered with kk (x3) fastest, then jj (x2).  The
    blocks are eliminated in ``order`` (``elimination_order``); when block i is eliminated,
    its Schur complement is S_i = K_ii - sum_j K_ij T_j K_ji over its already eliminated
    neighbours j, and ``block_T[i]`` = S_i^{-1} (numpy.linalg.inv: LU with partial pivoting
    inside the block; no pivoting across blocks).
    """

    def __init__(self, prob, Gz, zg, Gy, yg, order="up"):
        n, h = prob.n, prob.h
        zw0, zw1, zfirst, zlast = window_fronts(Gz, zg, prob.p, prob.fronts)
        yw0, yw1, yfirst, ylast = window_fronts(Gy, yg, prob.p, prob.fronts_inner)
        px = prob.boundary_axis()
        py = axis_profile(yw0, yw1, n, prob.b, prob.C, prob.omega, yfirst, prob.p, ylast, prob.C_mv)
        pz = axis_profile(zw0, zw1, n, prob.b, prob.C, prob.omega, zfirst, prob.p, zlast, prob.C_mv)
        K = assemble_box(prob.kappa[zw0 - 1:zw1, yw0 - 1:yw1, :], px, py, pz, h)
        self.Wy, self.Wz = yw1 - yw0 + 1, zw1 - zw0 + 1
        self.n, self.B = n, self.Wy * self.Wz
        self.K = K
        idx = np.arange(K.shape[0]).reshape(self.Wz, self.Wy, n)
        self.sel = [idx[:, :, i].T.ravel() for i in range(n)]   # unknowns of x1-block i
        self.order = elimination_order(n, order)
        # K_ij for neighbouring blocks (sparse)
        self.Kc = {}
        for i in range(n - 1):
            self.Kc[(i + 1, i)] = K[self.sel[i + 1]][:, self.sel[i]]
            self.Kc[(i, i + 1)] = K[self.sel[i]][:, self.sel[i + 1]]
        done = set()
        self.block_T = [None] * n
        for i in self.order:
            assert not (i - 1 in done and i + 1 in done and len(done) < n - 1), "not an end block"
            S = K[self.sel[i]][:, self.sel[i]].toarray()
            for j in (i - 1, i + 1):
                if j in done:
                    S = S - _dense_times_sparse(self.Kc[(i, j)] @ self.block_T[j], self.Kc[(j, i)])
            self.block_T[i] = np.linalg.inv(S)
            done.add(i)
        self.rank = {i: t for t, i in enumerate(self.order)}
        # line-grid unknowns of the physical rows (those of G_yg), in (kk, j, i) C-order
        a, e = Gy[yg]
        self.phys = idx[:, a - yw0:e - yw0 + 1, :].ravel()

    def _nbrs(self, i, before):
        """Neighbours of block i eliminated before (or after) it."""
        return [j for j in (i - 1, i + 1)
                if 0 <= j < self.n and (self.rank[j] < self.rank[i]) == before]

    def _solve(self, r, Kij, Ti):
        r = _cols(r)
        w = [r[s].astype(np.complex128) for s in self.sel]
        y = [None] * self.n
        for i in self.order:                              # L^{-1}, then diag(T)
            z = w[i]
            for j in self._nbrs(i, True):
                z = z - Kij(i, j) @ y[j]
            y[i] = Ti(i) @ z
        x = [None] * self.n
        for i in reversed(self.order):                    # U^{-1}
            c = 0
            for j in self._nbrs(i, False):
                c = c + Kij(i, j) @ x[j]
            x[i] = y[i] - Ti(i) @ c if not np.isscalar(c) else y[i]
        out = np.zeros(r.shape, np.complex128)
        for i, s in enumerate(self.sel):
            out[s] = x[i]
        return out

    def solve(self, r):
        """K^{-1} r through the factors (the solve formula of Sec. 3 / Sec. 4.1)."""
        return self._solve(r, lambda i, j: self.Kc[(i, j)], lambda i: self.block_T[i])

    def solve_adjoint(self, r):
        """K^{-H} r = L^{-H} D^{-H} U^{-H} r: the same passes with K^H and the T^H."""
        return self._solve(r, lambda i, j: self.Kc[(j, i)].conj().T,
                           lambda i: self.block_T[i].conj().T)


class SlabSweep:
    """Quasi-2D auxiliary problem of z-group zg and its inner sweep (Algorithms 3 and 4).

    Slab unknowns are ordered (kk, j, i) C-order, i.e. x1 fastest, over the z-window.
    """

    def __init__(self, prob, Gz, zg, Gy):
        n = prob.n
        zw0, zw1, zfirst, zlast = window_fronts(Gz, zg, prob.p, prob.fronts)
        ax = prob.boundary_axis()
        pz = axis_profile(zw0, zw1, n, prob.b, prob.C, prob.omega, zfirst, prob.p, zlast, prob.C_mv)
        self.H = assemble_box(prob.kappa[zw0 - 1:zw1], ax, ax, pz, prob.h)
        self.HH = self.H.conj().T.tocsr()
        self.Wz = zw1 - zw0 + 1
        idx = np.arange(self.H.shape[0]).reshape(self.Wz, n, n)
        self.rows = [idx[:, a - 1:e, :].ravel() for (a, e) in Gy]
        a, e = Gz[zg]
        self.phys = idx[a - zw0:e - zw0 + 1, :, :].ravel()
        self.fronts_inner = prob.fronts_inner
        self.lines = [LineFactors(prob, Gz, zg, Gy, yg) for yg in range(len(Gy))]  # Alg. 3

    def _line(self, yg, alpha, adjoint):
        """The approximate inverse of the line's block: embed, solve, restrict (Sec. 4.1)."""
        ln = self.lines[yg]
        r = np.zeros((ln.K.shape[0], alpha.shape[1]), np.complex128)
        r[ln.phys] = alpha
        x = ln.solve_adjoint(r) if adjoint else ln.solve(r)
        return x[ln.phys]

    def apply(self, gv, adjoint=False):
        """Algorithm 4: v ~ H^{-1} g (or the adjoint with H^H couplings and line adjoints).
        With two inner fronts the x2-groups are eliminated 0..mid-1, L-1..mid+1, mid (the same
        block order and couplings as the two-front outer sweep, one level down)."""
        H = self.HH if adjoint else self.H
        gv = _cols(gv)
        v = np.zeros(gv.shape, np.complex128)
        R = self.rows
        L = len(R)
        if self.fronts_inner == 2:
            blk = lambda a, b: H[R[a]][:, R[b]]
            mid = L // 2
            for yg in range(mid):
                rhs = gv[R[yg]].astype(np.complex128)
                if yg > 0:
                    rhs = rhs - blk(yg, yg - 1) @ v[R[yg - 1]]
                v[R[yg]] = self._line(yg, rhs, adjoint)
            for yg in range(L - 1, mid, -1):
                rhs = gv[R[yg]].astype(np.complex128)
                if yg < L - 1:
                    rhs = rhs - blk(yg, yg + 1) @ v[R[yg + 1]]
                v[R[yg]] = self._line(yg, rhs, adjoint)
            rhs = gv[R[mid]] - blk(mid, mid - 1) @ v[R[mid - 1]] - blk(mid, mid + 1) @ v[R[mid + 1]]
            v[R[mid]] = self._line(mid, rhs, adjoint)
            for yg in range(mid - 1, -1, -1):
                v[R[yg]] = v[R[yg]] - self._line(yg, blk(yg, yg + 1) @ v[R[yg + 1]], adjoint)
            for yg in range(mid + 1, L):
                v[R[yg]] = v[R[yg]] - self._line(yg, blk(yg, yg - 1) @ v[R[yg - 1]], adjoint)
            return v
        for yg in range(L):
            rhs = gv[R[yg]].astype(np.complex128)
            if yg > 0:
                rhs = rhs - H[R[yg]][:, R[yg - 1]] @ v[R[yg - 1]]
            v[R[yg]] = self._line(yg, rhs, adjoint)
        for yg in range(L - 2, -1, -1):
            v[R[yg]] = v[R[yg]] - self._line(yg, H[R[yg]][:, R[yg + 1]] @ v[R[yg + 1]], adjoint)
        return v


class RecursiveSweep:
    """Algorithm 5 (setup) and Algorithm 6 (apply) of Sec. 4.2; ``apply(.., adjoint=True)``
    gives M^{-H} (module docstring).  Vectors are ordered x1 fastest (Sec. 3).

    With ``prob.fronts == 2`` the outer sweep runs from both x3-faces (Sec. 4.2 note 3, the
    configuration of Sec. 5): the block LDU of Algorithm 6 with the x3-groups eliminated in
    the order 0..mid-1 (upwards), G-1..mid+1 (downwards), mid, each Schur complement replaced
    by the auxiliary problem padded on its eliminated side(s) (``partition.window_fronts``);
    forward, the two fronts carry f - A u from their eliminated neighbour and the middle group
    takes both; backward, each front subtracts the correction from the neighbour nearer the
    middle.  The inner sweep is Algorithm 4 from the x2 = 0 face, or with
    ``prob.fronts_inner == 2`` from both x2-faces in the same block order one level down
    (``SlabSweep.apply``), independently of the outer choice."""

    def __init__(self, prob):
        self.prob = prob
        n = prob.n
        self.Gz = (groups_two_fronts(n, prob.b, prob.d) if prob.fronts == 2
                   else groups(n, prob.first_z, prob.d))
        self.Gy = (groups_two_fronts(n, prob.b, prob.d) if prob.fronts_inner == 2
                   else groups(n, prob.first_y, prob.d))
        self.A = helmholtz_matrix(prob)
        self.AH = self.A.conj().T.tocsr()
        idx = np.arange(n ** 3).reshape(n, n, n)
        self.layers = [idx[a - 1:e].ravel() for (a, e) in self.Gz]
        self.slabs = [SlabSweep(prob, self.Gz, g, self.Gy) for g in range(len(self.Gz))]

    def _TT(self, g, alpha, adjoint):
        """The approximate inverse of the slab block: embed into the window, Algorithm 4, restrict."""
        s = self.slabs[g]
        gv = np.zeros((s.H.shape[0], alpha.shape[1]), np.complex128)
        gv[s.phys] = alpha
        return s.apply(gv, adjoint)[s.phys]

    def apply(self, f, adjoint=False):
        if self.prob.fronts == 2:
            return self._apply_two_fronts(f, adjoint)
        A = self.AH if adjoint else self.A
        f = _cols(f)
        u = np.zeros(f.shape, np.complex128)
        Ls = self.layers
        G = len(Ls)
        for g in range(G):
            rhs = f[Ls[g]].astype(np.complex128)
            if g > 0:
                rhs = rhs - A[Ls[g]][:, Ls[g - 1]] @ u[Ls[g - 1]]
            u[Ls[g]] = self._TT(g, rhs, adjoint)
        for g in range(G - 2, -1, -1):
            u[Ls[g]] = u[Ls[g]] - self._TT(g, A[Ls[g]][:, Ls[g + 1]] @ u[Ls[g + 1]], adjoint)
        return u

    def _apply_two_fronts(self, f, adjoint):
        A = self.AH if adjoint else self.A
        f = _cols(f)
        u = np.zeros(f.shape, np.complex128)
        Ls = self.layers
        G = len(Ls)
        mid = G // 2
        blk = lambda g, h: A[Ls[g]][:, Ls[h]]
        for g in range(mid):                              # front from x3 = 0, upwards
            rhs = f[Ls[g]].astype(np.complex128)
            if g > 0:
                rhs = rhs - blk(g, g - 1) @ u[Ls[g - 1]]
            u[Ls[g]] = self._TT(g, rhs, adjoint)
        for g in range(G - 1, mid, -1):                   # front from x3 = 1, downwards
            rhs = f[Ls[g]].astype(np.complex128)
            if g < G - 1:
                rhs = rhs - blk(g, g + 1) @ u[Ls[g + 1]]
            u[Ls[g]] = self._TT(g, rhs, adjoint)
        rhs = (f[Ls[mid]] - blk(mid, mid - 1) @ u[Ls[mid - 1]]
               - blk(mid, mid + 1) @ u[Ls[mid + 1]])      # the middle group, both sides
        u[Ls[mid]] = self._TT(mid, rhs, adjoint)
        for g in range(mid - 1, -1, -1):
            u[Ls[g]] = u[Ls[g]] - self._TT(g, blk(g, g + 1) @ u[Ls[g + 1]], adjoint)
        for g in range(mid + 1, G):
            u[Ls[g]] = u[Ls[g]] - self._TT(g, blk(g, g - 1) @ u[Ls[g - 1]], adjoint)
        return u

    def lines(self):
        """(zg, yg, LineFactors) in sweep order: z-group major, y-group minor."""
        for g, s in enumerate(self.slabs):
            for l, ln in enumerate(s.lines):
                yield g, l, ln
