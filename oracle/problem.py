"""Sec. 2 of the paper: the PML profiles and the 7-point discretisation, eq. (3).

Test infrastructure only (see ``oracle/__init__.py``).

Positions along an axis are handled as integer *half-steps* t: the position is t*h/2, so
node m is t = 2m and the half-node m - 1/2 is t = 2m - 1.  This keeps every "is this
point below the first physical node" decision exact.

Pins (tests/test_oracle_operator.py): with sigma = 0 the assembled operator has the
closed-form sine eigenpairs of the 7-point Laplacian; with a PML it converges to the
continuous operator sum_d s_d d/dx_d (s_d d/dx_d) + omega^2/c^2; each directional part
divided row-wise by its s_d at the node is complex symmetric; a 1D PML-padded problem
reproduces the outgoing 1D Green's function.
"""
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import scipy.sparse as sp


def sigma(xi, eta, C):
    """Damping profile of Sec. 2: (C/eta) * ((xi - eta)/eta)^2 for xi in [0, eta], else 0."""
    xi = np.asarray(xi, dtype=np.float64)
    val = (C / eta) * ((xi - eta) / eta) ** 2
    return np.where((xi >= 0.0) & (xi <= eta), val, 0.0)


def stretch(sig, omega):
    """Complex stretching s = (1 + i sigma/omega)^(-1) of Sec. 2."""
    return 1.0 / (1.0 + 1j * np.asarray(sig, dtype=np.float64) / omega)


def boundary_profile(t, n, b, C, omega):
    """s of the boundary PML at half-step positions t (position t*h/2, h = 1/(n+1)).

    Sec. 2 puts a PML of width eta = b*h at x = 0; the experiments of Sec. 5 put PMLs on all
    six faces, so the damping is mirrored: sigma(x) + sigma(1 - x).
    """
    h = 1.0 / (n + 1)
    eta = b * h
    t = np.asarray(t, dtype=np.float64)
    x_lo = 0.5 * t * h
    x_hi = 0.5 * (2 * (n + 1) - t) * h          # 1 - x, computed from integers
    return stretch(sigma(x_lo, eta, C) + sigma(x_hi, eta, C), omega)


def moving_profile(t, first_phys, p, n, C, omega):
    """s of a moving PML of p cells placed right below node ``first_phys`` (Sec. 3, domain D_m).

    The auxiliary problem has its zero-Dirichlet plane p+1 spacings below the first physical
    node, and the damping sigma(xi; eta=(p+1)h) is measured from that plane, so all p padded
    nodes are damped and the first physical node is not.  For one physical layer and p = b-1
    this is exactly D_m = [(m-b)h, (m+1)h] with s(x - (m-b)h).
    """
    h = 1.0 / (n + 1)
    xi = 0.5 * (np.asarray(t, dtype=np.float64) - 2 * (first_phys - p - 1)) * h
    return stretch(sigma(xi, (p + 1) * h, C), omega)


def moving_profile_above(t, last_phys, p, n, C, omega):
    """Mirror image of ``moving_profile``: a moving PML of p cells right above node
    ``last_phys``, its zero-Dirichlet plane p+1 spacings above that node (the auxiliary
    problems of a front sweeping from x = 1 downwards, Sec. 4.2 note on PML on all faces)."""
    h = 1.0 / (n + 1)
    xi = 0.5 * (2 * (last_phys + p + 1) - np.asarray(t, dtype=np.float64)) * h
    return stretch(sigma(xi, (p + 1) * h, C), omega)


@dataclass
class AxisProfile:
    """s along one axis of a window [w0, w1] (1-based global node indices).

    ``node[a]`` is s at node w0+a; ``half[a]`` is s at the half-node w0+a-1/2, so node a
    sits between ``half[a]`` (below) and ``half[a+1]`` (above).
    """
    w0: int
    w1: int
    node: np.ndarray
    half: np.ndarray


def axis_profile(w0, w1, n, b, C, omega, first_phys=None, p=0, last_phys=None, C_mv=None):
    """Profile of a window.  With ``first_phys`` set, positions strictly below that node use
    the moving PML (the auxiliary profile replaces the original one there, Sec. 3 and 4.1);
    with ``last_phys`` set, positions strictly above that node use the mirrored moving PML;
    all other positions keep the boundary profile, including the far-face PML.  The moving
    PML takes the constant C_mv (default C)."""
    Cm = C if C_mv is None else C_mv
    m = np.arange(w0, w1 + 1)
    t_node = 2 * m
    t_half = 2 * np.arange(w0, w1 + 2) - 1
    node = boundary_profile(t_node, n, b, C, omega)
    half = boundary_profile(t_half, n, b, C, omega)
    if first_phys is not None:
        below_n = t_node < 2 * first_phys
        below_h = t_half < 2 * first_phys
        node = np.where(below_n, moving_profile(t_node, first_phys, p, n, Cm, omega), node)
        half = np.where(below_h, moving_profile(t_half, first_phys, p, n, Cm, omega), half)
    if last_phys is not None:
        above_n = t_node > 2 * last_phys
        above_h = t_half > 2 * last_phys
        node = np.where(above_n, moving_profile_above(t_node, last_phys, p, n, Cm, omega), node)
        half = np.where(above_h, moving_profile_above(t_half, last_phys, p, n, Cm, omega), half)
    return AxisProfile(w0, w1, node, half)


def assemble_box(kappa, px, py, pz, h, parts=False):
    """Eq. (3) on a box of nodes with zero Dirichlet data outside it.

    ``kappa`` has shape (nz, ny, nx) (x3, x2, x1); unknowns are ordered x1 fastest, then x2,
    then x3 (the column-major order of Sec. 3).  Row of node p, direction d:
      (s_d)_p / h * [ (s_d)_{p+e_d/2}/h (u_{p+e_d} - u_p) - (s_d)_{p-e_d/2}/h (u_p - u_{p-e_d}) ]
    plus kappa_p u_p.  Neighbours outside the box are zero (Dirichlet), but their
    coefficient still enters the diagonal.

    With ``parts=True`` returns (A, {"x": A1, "y": A2, "z": A3, "k": diag(kappa)}).
    """
    kappa = np.asarray(kappa)
    nz, ny, nx = kappa.shape
    N = nx * ny * nz
    idx = np.arange(N).reshape(nz, ny, nx)
    pieces = {}
    for name, axis, prof in (("x", 2, px), ("y", 1, py), ("z", 0, pz)):
        L = kappa.shape[axis]
        assert prof.node.shape == (L,) and prof.half.shape == (L + 1,)
        shape = [1, 1, 1]
        shape[axis] = L
        s_node = prof.node.reshape(shape)
        c_up = np.broadcast_to(s_node * prof.half[1:].reshape(shape) / h ** 2, kappa.shape)
        c_dn = np.broadcast_to(s_node * prof.half[:-1].reshape(shape) / h ** 2, kappa.shape)
        lo = [slice(None)] * 3
        hi = [slice(None)] * 3
        lo[axis] = slice(0, L - 1)
        hi[axis] = slice(1, L)
        lo, hi = tuple(lo), tuple(hi)
        rows = np.concatenate([idx[lo].ravel(), idx[hi].ravel(), idx.ravel()])
        cols = np.concatenate([idx[hi].ravel(), idx[lo].ravel(), idx.ravel()])
        vals = np.concatenate([c_up[lo].ravel(), c_dn[hi].ravel(), -(c_up + c_dn).ravel()])
        pieces[name] = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    pieces["k"] = sp.diags(kappa.astype(np.complex128).ravel()).tocsr()
    A = (pieces["x"] + pieces["y"] + pieces["z"] + pieces["k"]).tocsr()
    return (A, pieces) if parts else A


@dataclass
class Problem:
    """One instance of eq. (3) plus the sweep parameters.

    n: interior nodes per axis (h = 1/(n+1)); c: velocity at the nodes, shape (n, n, n)
    indexed [k, j, i] (x3, x2, x1); omega; b: boundary PML cells (eta = b h); C: the constant
    of sigma; p: moving-PML cells; d: physical layers per auxiliary problem (same in x2 and
    x3); first_y / first_z: size of the first group along x2 / x3 (b by default; other
    values only serve the degenerate-partition pins); fronts: 1 for the single-front outer
    sweep of Algorithm 6, 2 for the outer sweep from both x3-faces meeting in a middle slab
    (the configuration of the paper's experiments, Sec. 4.2 note 3 and Sec. 5); fronts_inner:
    the same choice for the inner sweep over x2 (Algorithm 4); C_moving: the constant of the
    auxiliary problems' moving PML (0: C).  The paper fixes neither constant; only C enters
    eq. (3) itself.
    """
    n: int
    c: np.ndarray
    omega: float
    b: int
    C: float
    p: int
    d: int = 1
    first_y: Optional[int] = None
    first_z: Optional[int] = None
    fronts: int = 1
    fronts_inner: int = 1
    C_moving: float = 0.0
    h: float = field(init=False)

    def __post_init__(self):
        self.h = 1.0 / (self.n + 1)
        self.c = np.asarray(self.c, dtype=np.float64)
        assert self.c.shape == (self.n,) * 3
        if self.first_y is None:
            self.first_y = self.b
        if self.first_z is None:
            self.first_z = self.b

    @property
    def C_mv(self):
        return self.C_moving if self.C_moving > 0 else self.C

    @property
    def kappa(self):
        """(omega^2 / c^2) at the nodes, the zeroth-order coefficient of eq. (3)."""
        return self.omega ** 2 / self.c ** 2

    def boundary_axis(self):
        return axis_profile(1, self.n, self.n, self.b, self.C, self.omega)


def helmholtz_matrix(prob, parts=False):
    """The full system matrix A of eq. (3) on the interior grid P (Sec. 2)."""
    ax = prob.boundary_axis()
    return assemble_box(prob.kappa, ax, ax, ax, prob.h, parts=parts)
