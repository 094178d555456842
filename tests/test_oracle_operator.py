"""Pins of the oracle's PML profiles and 7-point operator (Sec. 2, eq. (3)) against facts
that do not come from the oracle itself."""
import numpy as np
import pytest

import oracle as O
from oracle.problem import AxisProfile


def _unit_axis(L):
    return AxisProfile(1, L, np.ones(L, complex), np.ones(L + 1, complex))


def test_sigma_and_stretch_shape():
    # sigma vanishes at eta and beyond, is C/eta at 0 and decreases quadratically in between
    eta, C = 0.25, 7.0
    xs = np.array([0.0, eta / 2, eta, 0.5, 1.0])
    s = O.sigma(xs, eta, C)
    assert s[0] == pytest.approx(C / eta)
    assert s[1] == pytest.approx(C / eta / 4)
    assert s[2] == 0 and s[3] == 0 and s[4] == 0
    # s = 1/(1 + i sigma/omega): |s| <= 1 and Im s <= 0 when sigma >= 0 (outgoing stretching)
    st = O.stretch(O.sigma(np.linspace(0, 1, 41), eta, C), 10.0)
    assert np.all(np.abs(st) <= 1 + 1e-15) and np.all(st.imag <= 0)


def test_laplacian_sine_eigenpairs():
    """With sigma = 0 (s = 1) eq. (3) is the 7-point Laplacian plus kappa; products of sines are
    eigenvectors with eigenvalue kappa - 4/h^2 sum_d sin^2(pi m_d h / 2)."""
    nx, ny, nz = 7, 5, 6
    h = 0.1
    kap = 3.5
    A = O.assemble_box(np.full((nz, ny, nx), kap), _unit_axis(nx), _unit_axis(ny), _unit_axis(nz), h)
    # a box of nx nodes with Dirichlet ends has sine modes sin(pi a i/(nx+1))
    for (a, b_, c) in [(1, 1, 1), (2, 3, 1), (7, 5, 6), (4, 2, 5)]:
        i = np.arange(1, nx + 1)
        j = np.arange(1, ny + 1)
        k = np.arange(1, nz + 1)
        v = (np.sin(np.pi * c * k / (nz + 1))[:, None, None] * np.sin(np.pi * b_ * j / (ny + 1))[None, :, None]
             * np.sin(np.pi * a * i / (nx + 1))[None, None, :]).ravel()
        lam = kap - 4 / h ** 2 * (np.sin(np.pi * a / (2 * (nx + 1))) ** 2 + np.sin(np.pi * b_ / (2 * (ny + 1))) ** 2
                                  + np.sin(np.pi * c / (2 * (nz + 1))) ** 2)
        assert np.linalg.norm(A @ v - lam * v) <= 1e-12 * abs(lam) * np.linalg.norm(v)


def test_directional_parts_symmetric_after_row_scaling():
    """Each directional part of eq. (3) is diag(s_d at nodes) times a complex-symmetric matrix
    (the flux form (s_d/h)[(s_d)_{+1/2}/h .. - (s_d)_{-1/2}/h ..])."""
    n, b = 9, 3
    prob = O.Problem(n=n, c=1 + 0.1 * np.random.default_rng(0).random((n, n, n)), omega=20.0, b=b, C=90.0, p=3)
    A, parts = O.helmholtz_matrix(prob, parts=True)
    ax = prob.boundary_axis()
    s = ax.node
    for name, axis in (("x", 2), ("y", 1), ("z", 0)):
        shape = [1, 1, 1]
        shape[axis] = n
        sd = np.broadcast_to(s.reshape(shape), (n, n, n)).ravel()
        Ssym = (parts[name].multiply(1.0 / sd[:, None])).tocsr()
        assert abs(Ssym - Ssym.T).max() <= 1e-9 * abs(Ssym).max()
    # the non-symmetric form: A itself is not symmetric when the PML is on
    assert abs(A - A.T).max() > 1e-3 * abs(A).max()


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_consistency_with_continuous_pml_operator(axis):
    """For smooth u, (A u)_p approaches [sum_d s_d d/dx_d (s_d du/dx_d) + kappa u](p) as h -> 0.
    sigma is C^1 with a jump in its second derivative at eta, so the max error decays at least
    like h there and like h^2 elsewhere; a dropped term, wrong sign or swapped half-node gives
    an O(1) error instead."""
    errs = []
    for n in (23, 47, 95):
        h = 1.0 / (n + 1)
        b = (n + 1) // 4              # eta = 1/4 at every resolution
        C, om = 3.0, 5.0
        x = np.arange(1, n + 1) * h
        prof = O.axis_profile(1, n, n, b, C, om)
        flat = _unit_axis(n)
        profs = [flat, flat, flat]
        profs[2 - axis] = prof      # axis 0 -> z, 2 -> x
        # 1D test: u depends on the profiled coordinate only, other directions have one node
        shape = [1, 1, 1]
        shape[axis] = n
        kap = np.full(shape, 2.0)
        single = AxisProfile(1, 1, np.ones(1, complex), np.ones(2, complex))
        pp = [single, single, single]
        pp[2 - axis] = prof
        A, parts = O.assemble_box(kap, pp[0], pp[1], pp[2], h, parts=True)
        Ad = parts["xyz"[2 - axis]] + parts["k"]
        u = np.sin(np.pi * x) ** 2 * np.cos(3 * x)
        up = 2 * np.pi * np.sin(np.pi * x) * np.cos(np.pi * x) * np.cos(3 * x) - 3 * np.sin(np.pi * x) ** 2 * np.sin(3 * x)
        upp = (2 * np.pi ** 2 * np.cos(2 * np.pi * x) * np.cos(3 * x) - 6 * np.pi * np.sin(2 * np.pi * x) * np.sin(3 * x)
               - 9 * np.sin(np.pi * x) ** 2 * np.cos(3 * x))
        eta = b * h
        sig = O.sigma(x, eta, C) + O.sigma(1 - x, eta, C)
        dsig = np.where(x <= eta, -2 * C / eta ** 3 * (eta - x), 0.0) + np.where(1 - x <= eta, 2 * C / eta ** 3 * (eta - (1 - x)), 0.0)
        s = 1 / (1 + 1j * sig / om)
        ds = -(1j * dsig / om) * s ** 2
        cont = s * (ds * up + s * upp) + 2.0 * u
        errs.append(np.max(np.abs(Ad @ u - cont)) / np.max(np.abs(cont)))
    assert errs[0] / errs[1] > 1.8 and errs[1] / errs[2] > 1.8, errs
    assert errs[2] < 0.01, errs


def test_1d_pml_reproduces_discrete_outgoing_green_function():
    """A 1D line padded with the boundary PML on both ends: away from the PML the discrete
    solution of (s(s u')')' + k^2 u = delta/h equals the closed-form outgoing discrete Green's
    function h e^{i theta |i-i0|} / (2 i sin theta), cos theta = 1 - k^2 h^2 / 2, up to the
    PML's reflection."""
    n, b = 399, 60
    h = 1.0 / (n + 1)
    k = 2 * np.pi / (10 * h)                 # 10 points per wavelength
    C = 30.0 * b
    prof = O.axis_profile(1, n, n, b, C, k)
    single = AxisProfile(1, 1, np.ones(1, complex), np.ones(2, complex))
    A, parts = O.assemble_box(np.full((1, 1, n), k ** 2), prof, single, single, h, parts=True)
    A1 = (parts["x"] + parts["k"]).tocsc()
    i0 = (n + 1) // 2
    f = np.zeros(n, complex)
    f[i0 - 1] = 1.0 / h
    import scipy.sparse.linalg as spla
    u = spla.spsolve(A1, f)
    theta = np.arccos(1 - k ** 2 * h ** 2 / 2)
    i = np.arange(1, n + 1)
    G = h * np.exp(1j * theta * np.abs(i - i0)) / (2j * np.sin(theta))
    inner = (i > b + 5) & (i < n - b - 5)
    assert np.max(np.abs(u[inner] - G[inner])) < 1e-3 * np.max(np.abs(G))
    # the wrong-sign stretching would be an incoming (growing) wave: make sure the test sees it
    prof_bad = O.axis_profile(1, n, n, b, -C, k)
    A_bad, pb = O.assemble_box(np.full((1, 1, n), k ** 2), prof_bad, single, single, h, parts=True)
    u_bad = spla.spsolve((pb["x"] + pb["k"]).tocsc(), f)
    assert np.max(np.abs(u_bad[inner] - G[inner])) > 0.1 * np.max(np.abs(G))


@pytest.mark.slow
def test_free_space_green_function_3d():
    """Constant c = 1, PML on all faces (c1-like at n = 23): the discrete solution for a unit
    point source approaches the outgoing free-space Green's function -e^{i omega r}/(4 pi r)
    (the equation is Laplace(u) + k^2 u = f, so the sign is negative).  At 8 points per
    wavelength the 7-point dispersion error is ~10-20 % on the shell, so the bound is loose;
    a conjugated (incoming) or mis-normalised solution is far outside it."""
    import scipy.sparse.linalg as spla
    n, b = 23, 5
    h = 1.0 / (n + 1)
    om = 2 * np.pi / (8 * h)
    prob = O.Problem(n=n, c=np.ones((n, n, n)), omega=om, b=b, C=30.0 * b, p=b)
    A = O.helmholtz_matrix(prob)
    m = (n + 1) // 2
    f = np.zeros((n, n, n), complex)
    f[m - 1, m - 1, m - 1] = 1 / h ** 3
    u = spla.spsolve(A.tocsc(), f.ravel()).reshape(n, n, n)
    K, J, I = np.meshgrid(*(np.arange(1, n + 1),) * 3, indexing="ij")
    r = h * np.sqrt((I - m) ** 2 + (J - m) ** 2 + (K - m) ** 2)
    G = -np.exp(1j * om * np.maximum(r, 1e-9)) / (4 * np.pi * np.maximum(r, 1e-9))
    shell = (r >= 3 * h) & (r <= 0.25)
    err = np.linalg.norm(u[shell] - G[shell]) / np.linalg.norm(G[shell])
    err_conj = np.linalg.norm(np.conj(u[shell]) - G[shell]) / np.linalg.norm(G[shell])
    assert err < 0.3 and err_conj > 1.0
