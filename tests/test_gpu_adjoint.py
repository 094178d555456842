"""GPU parity of the adjoint path (row a11): M^{-H} and A^H dot tests, adjoint solves, the
misfit/adjoint-source kernel, the velocity gradient against the oracle's adjoint-state
gradient, and the autograd wrapper against central differences of the GPU misfit.

Tolerances: complex128 dot tests 1e-12 (rounding); gradients from solves at tol 1e-10 agree
with the oracle's sparse-direct gradient to 1e-6 relative (the solve tolerance times the
conditioning of the adjoint pair); complex64 sweeps inside FP64 FGMRES reach the same
residuals, so the mixed gradient error is of the same order (stated in the test output)."""
import numpy as np
import pytest

import oracle as O
from paper_1502_07266_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N, BW = 13, 3


def _case():
    sc = inputs.small_case(n=N, b=BW, p=BW)
    prob = O.Problem(n=N, c=sc["c"], omega=sc["omega"], b=BW, C=sc["C"], p=BW)
    return sc, prob


def _helm(sc, prec):
    from paper_1502_07266_amd.binding import Helm
    return Helm(torch.from_numpy(sc["c"]).cuda(), sc["omega"], BW, sc["C"], BW, 1, prec=prec)


def _gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("prec,tol", [("c128", 1e-12), ("c64", 2e-5)])
def test_adjoint_dot_tests(prec, tol):
    sc, prob = _case()
    H = _helm(sc, prec)
    x, y = inputs.random_rhs(N, 2, seed=31)
    X, Y = _gpu(x), _gpu(y)
    mx = H.apply(X)[0].cpu().numpy()
    mhy = H.apply(Y, adjoint=True)[0].cpu().numpy()
    d1, d2 = np.vdot(mx, y), np.vdot(x, mhy)
    assert abs(d1 - d2) <= tol * abs(d1)
    ax = H.matvec(X)[0].cpu().numpy()
    ahy = H.matvec(Y, adjoint=True)[0].cpu().numpy()
    assert abs(np.vdot(ax, y) - np.vdot(x, ahy)) <= 1e-12 * abs(np.vdot(ax, y))


@pytest.mark.parametrize("prec", ["c128", "c64"])
def test_adjoint_solve(prec):
    import scipy.sparse.linalg as spla
    sc, prob = _case()
    H = _helm(sc, prec)
    f = inputs.random_rhs(N, 2, seed=32)
    u, its, rel, rc = H.solve(_gpu(f), tol=1e-9, adjoint=True)
    AH = O.helmholtz_matrix(prob).conj().T.tocsc()
    ref = spla.spsolve(AH, f.reshape(2, -1).T).T.reshape(f.shape)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    print(f"adjoint solve {prec}: its {its} err {err:.2e}")
    assert rc == 0 and err <= 1e-7


def _data(sc, prob):
    nodes = [(5, 7, BW + 1), (8, 6, BW + 2)]
    F = inputs.sources(N, nodes)
    plane = N - BW
    prob0 = O.Problem(n=N, c=np.full((N, N, N), 1.15), omega=prob.omega, b=BW, C=prob.C, p=BW)
    _, _, U0 = O.misfit_and_gradient(prob0, F, plane, np.zeros((2, N, N)))
    return F, plane, U0[:, plane - 1]


def test_misfit_kernel():
    sc, prob = _case()
    H = _helm(sc, "c128")
    F, plane, d_obs = _data(sc, prob)
    u = inputs.random_rhs(N, 2, seed=33)
    J, g = H.misfit(_gpu(u), _gpu(d_obs), plane)
    res = u[:, plane - 1] - d_obs
    assert abs(J - 0.5 * np.sum(np.abs(res) ** 2)) <= 1e-12 * J
    g = g.cpu().numpy()
    assert np.array_equal(g[:, plane - 1], res)
    mask = np.ones(N, bool)
    mask[plane - 1] = False
    assert not np.any(g[:, mask])


@pytest.mark.parametrize("prec,tol", [("c128", 1e-6), ("c64", 1e-6)])
def test_gradient_matches_oracle(prec, tol):
    from paper_1502_07266_amd.autograd import misfit
    sc, prob = _case()
    F, plane, d_obs = _data(sc, prob)
    J_ref, g_ref, _ = O.misfit_and_gradient(prob, F, plane, d_obs)
    c = torch.from_numpy(sc["c"]).cuda().requires_grad_(True)
    J = misfit(c, _gpu(F), _gpu(d_obs), plane, omega=sc["omega"], b=BW, C=sc["C"], p=BW,
               prec=prec, tol=1e-10)
    J.backward()
    g = c.grad.cpu().numpy()
    eJ = abs(J.item() - J_ref) / J_ref
    eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    print(f"gradient {prec}: J rel err {eJ:.2e}, grad rel err {eg:.2e}")
    assert eJ <= tol and eg <= tol


def test_autograd_against_central_differences():
    """Central differences of the GPU misfit (FP64 solves at tol 1e-12, step 1e-4) at seeded
    non-PML cells agree with the adjoint gradient."""
    from paper_1502_07266_amd.autograd import misfit
    sc, prob = _case()
    F, plane, d_obs = _data(sc, prob)
    kw = dict(omega=sc["omega"], b=BW, C=sc["C"], p=BW, prec="c128", tol=1e-12)
    c0 = torch.from_numpy(sc["c"]).cuda()
    c = c0.clone().requires_grad_(True)
    J = misfit(c, _gpu(F), _gpu(d_obs), plane, **kw)
    J.backward()
    g = c.grad.cpu().numpy()
    eps = 1e-4
    for (i, j, k) in inputs.fd_cells(N, BW, 4):
        cp, cm = c0.clone(), c0.clone()
        cp[k - 1, j - 1, i - 1] += eps
        cm[k - 1, j - 1, i - 1] -= eps
        with torch.no_grad():
            Jp = misfit(cp, _gpu(F), _gpu(d_obs), plane, **kw).item()
            Jm = misfit(cm, _gpu(F), _gpu(d_obs), plane, **kw).item()
        fd = (Jp - Jm) / (2 * eps)
        assert abs(fd - g[k - 1, j - 1, i - 1]) <= 1e-5 * max(abs(fd), 1e-3 * np.abs(g).max()), ((i, j, k), fd, g[k - 1, j - 1, i - 1])
