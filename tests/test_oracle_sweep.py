"""Pins of the oracle's recursive sweep (Sec. 3-4, Algorithms 3-6) against exact solves,
the non-recursive Algorithm 2 with exact auxiliary solves, the exact block LDU of Sec. 3,
and linear-algebra invariants."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from oracle.reference import nonrecursive_apply, exact_layer_T
from oracle.partition import groups, window
from oracle.problem import axis_profile, assemble_box
from paper_1502_07266_amd import inputs


def _prob(n=11, b=3, p=3, d=1, **kw):
    case = inputs.small_case(n=n, b=b, p=p, d=d)
    return O.Problem(n=n, c=case["c"], omega=case["omega"], b=b, C=case["C"], p=p, d=d, **kw)


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def test_groups_and_windows():
    G = groups(20, 4, 3)
    assert G == [(1, 4), (5, 7), (8, 10), (11, 13), (14, 16), (17, 19), (20, 20)]
    assert window(G, 0, 2) == (1, 4, None)
    assert window(G, 1, 2) == (3, 7, 5)
    assert window(G, 6, 4) == (16, 20, 20)


def test_moving_profile_matches_shifted_boundary_profile():
    """For one physical layer and p = b-1 the moving profile is the paper's s(x3 - (m-b)h) on
    D_m = [(m-b)h, (m+1)h] (Sec. 3), i.e. the boundary profile of width b h shifted."""
    n, b, C, om = 30, 5, 150.0, 12.0
    h = 1 / (n + 1)
    m = 17
    prof = axis_profile(m - (b - 1), m, n, b, C, om, first_phys=m, p=b - 1)
    xs_node = np.arange(m - b + 1, m + 1) * h - (m - b) * h
    xs_half = (np.arange(m - b + 1, m + 2) - 0.5) * h - (m - b) * h
    s = lambda x: 1 / (1 + 1j * O.sigma(x, b * h, C) / om)
    assert np.allclose(prof.node, s(xs_node), rtol=1e-14, atol=0)
    # the half-node above the physical layer keeps the boundary profile (undamped here)
    assert np.allclose(prof.half[:-1], s(xs_half[:-1]), rtol=1e-14, atol=0)
    assert prof.half[-1] == 1.0


@pytest.mark.parametrize("order", ["up", "down", "two-sided"])
def test_line_ldu_reproduces_line_matrix_and_dense_solve(order):
    prob = _prob(n=9, b=3, p=2)
    M = O.RecursiveSweep(prob)
    rng = np.random.default_rng(5)
    checked = 0
    for g, l, _ in M.lines():
        if (g, l) not in [(0, 0), (0, 2), (2, 0), (3, 4), (6, 6)]:
            continue
        ln = O.LineFactors(prob, M.Gz, g, M.Gy, l, order=order)
        K = ln.K.toarray()
        Nl = K.shape[0]
        # K with its blocks in elimination order equals Lc Uc: Lc has the diagonal blocks
        # S_i = T_i^{-1} and K_ij below it (j eliminated before i), Uc is unit upper with T_j K_ji
        B, n = ln.B, ln.n
        pos = {i: t for t, i in enumerate(ln.order)}
        perm = np.concatenate([ln.sel[i] for i in ln.order])
        Kb = K[np.ix_(perm, perm)]
        Lc = np.zeros_like(Kb)
        Uc = np.eye(Nl, dtype=complex)
        blk = lambda i: slice(pos[i] * B, (pos[i] + 1) * B)
        for i in range(n):
            Lc[blk(i), blk(i)] = np.linalg.inv(ln.block_T[i])
            for j in (i - 1, i + 1):
                if 0 <= j < n and pos[j] < pos[i]:
                    Lc[blk(i), blk(j)] = ln.Kc[(i, j)].toarray()
                    Uc[blk(j), blk(i)] = ln.block_T[j] @ ln.Kc[(j, i)].toarray()
        assert np.linalg.norm(Lc @ Uc - Kb) <= 1e-12 * np.linalg.norm(Kb)
        r = rng.standard_normal((Nl, 2)) + 1j * rng.standard_normal((Nl, 2))
        assert _rel(ln.solve(r), np.linalg.solve(K, r)) < 1e-12
        assert _rel(ln.solve_adjoint(r), np.linalg.solve(K.conj().T, r)) < 1e-12
        checked += 1
    assert checked == 5


@pytest.mark.parametrize("n", [9, 10])
def test_line_factor_ends_are_exact_blocks(n):
    """The first block eliminated has T = K_ii^{-1}; the last one has T = (K^{-1})_ii (its
    Schur complement is the whole matrix condensed onto it), in every elimination order."""
    prob = _prob(n=n, b=3, p=2)
    from oracle.partition import groups
    Gz = groups(prob.n, prob.b, prob.d)
    for (g, l) in [(0, 1), (2, 3), (4, 2)]:
        for order in ["up", "down", "two-sided"]:
            ln = O.LineFactors(prob, Gz, g, Gz, l, order=order)
            K = ln.K.toarray()
            Kinv = np.linalg.inv(K)
            first, last = ln.order[0], ln.order[-1]
            s0, s1 = ln.sel[first], ln.sel[last]
            assert np.allclose(ln.block_T[first], np.linalg.inv(K[np.ix_(s0, s0)]), rtol=1e-12, atol=0)
            ref = Kinv[np.ix_(s1, s1)]
            assert np.linalg.norm(ln.block_T[last] - ref) <= 1e-10 * np.linalg.norm(ref)
        two = O.elimination_order(n, "two-sided")
        m = n // 2
        assert two[-1] == m and sorted(two) == list(range(n))
        assert two[:m] == list(range(m)) and two[m:-1] == list(range(n - 1, m, -1))


def test_degenerate_single_groups_give_exact_inverse():
    """First group = whole axis in x2 and x3: one line problem equal to A, M^{-1} = A^{-1}."""
    n = 9
    prob = _prob(n=n, first_y=n, first_z=n)
    M = O.RecursiveSweep(prob)
    f = inputs.random_rhs(n, 2).reshape(2, -1).T
    x = spla.spsolve(M.A.tocsc(), f)
    assert _rel(M.apply(f), x) < 1e-12
    assert _rel(M.apply(f, adjoint=True), spla.spsolve(M.A.conj().T.tocsc(), f)) < 1e-12


@pytest.mark.parametrize("d", [1, 2])
def test_single_y_group_equals_nonrecursive_x3_sweep(d):
    """First x2-group = whole axis: each slab has one line = the whole quasi-2D problem, so
    Algorithm 6 is Algorithm 2 along x3 with exact auxiliary solves (d = 2 has a ragged
    last group since n - b is odd)."""
    n = 10
    prob = _prob(n=n, d=d, first_y=n)
    f = inputs.random_rhs(n, 2).reshape(2, -1).T
    assert _rel(O.RecursiveSweep(prob).apply(f), nonrecursive_apply(prob, f, "z")) < 1e-12


@pytest.mark.parametrize("d", [1, 2])
def test_single_z_group_equals_nonrecursive_x2_sweep(d):
    """First x3-group = whole axis: one slab = A, swept along x2 with exact quasi-1D solves,
    i.e. Algorithm 2 along x2 with exact auxiliary solves."""
    n = 10
    prob = _prob(n=n, d=d, first_z=n)
    f = inputs.random_rhs(n, 2).reshape(2, -1).T
    assert _rel(O.RecursiveSweep(prob).apply(f), nonrecursive_apply(prob, f, "y")) < 1e-12


def test_moving_pml_approximates_exact_schur_inverse():
    """T_m = S_m^{-1} of the exact layer LDU (Sec. 3) is the half-space Green's function on
    layer m; the auxiliary problem with a moving PML of p cells approximates it, better as p
    grows, and much better than the same window without damping.  (The floor of ~0.1 is the
    scattering by the medium below layer m, which the auxiliary problem drops.)"""
    n, b, m = 19, 5, 15
    case = inputs.small_case(n=n, b=b, p=b)
    prob = O.Problem(n=n, c=case["c"], omega=case["omega"], b=b, C=case["C"], p=b)
    Tex = exact_layer_T(prob)[m - 1]
    ax = prob.boundary_axis()
    errs = []
    for p, C in [(1, case["C"]), (2, case["C"]), (3, case["C"]), (4, case["C"]), (5, case["C"]), (5, 0.0)]:
        pz = axis_profile(m - p, m, n, b, C, prob.omega, first_phys=m, p=p)
        H = assemble_box(prob.kappa[m - p - 1:m], ax, ax, pz, prob.h).toarray()
        Hinv = np.linalg.inv(H)
        last = slice(p * n * n, (p + 1) * n * n)
        errs.append(np.linalg.norm(Hinv[last, last] - Tex) / np.linalg.norm(Tex))
    assert errs[0] > errs[1] > errs[2] > errs[3] > errs[4], errs
    assert errs[4] < 0.2 and errs[5] > 3 * errs[4], errs


def test_preconditioner_linear_and_adjoint_dot():
    prob = _prob(n=11)
    M = O.RecursiveSweep(prob)
    x, y = inputs.random_rhs(11, 2, seed=7).reshape(2, -1)
    a, bb = 0.3 - 1.1j, 2.0 + 0.5j
    lhs = M.apply(a * x + bb * y)[:, 0]
    rhs = a * M.apply(x)[:, 0] + bb * M.apply(y)[:, 0]
    assert _rel(lhs, rhs) < 1e-13
    d1 = np.vdot(M.apply(x)[:, 0], y)
    d2 = np.vdot(x, M.apply(y, adjoint=True)[:, 0])
    assert abs(d1 - d2) <= 1e-13 * abs(d1)
    d3 = np.vdot(M.A @ x, y)
    d4 = np.vdot(x, M.AH @ y)
    assert abs(d3 - d4) <= 1e-13 * abs(d3)


def test_preconditioner_is_close_to_inverse():
    """M^{-1} approximates A^{-1} well enough that GMRES converges in a handful of iterations
    (Sec. 5 reports 4-6 at 1e-3); here only that the preconditioned residual contracts."""
    prob = _prob(n=11)
    M = O.RecursiveSweep(prob)
    f = inputs.random_rhs(11, 1, seed=3).reshape(-1)
    x = spla.spsolve(M.A.tocsc(), f)
    z = M.apply(f)[:, 0]
    assert _rel(z, x) < 0.8
    assert np.linalg.norm(f - M.A @ z) < 0.8 * np.linalg.norm(f)


# ---------------------------------------------------------------------------------------
# two fronts in x3 (Sec. 4.2 note 3, Sec. 5)
# ---------------------------------------------------------------------------------------
from oracle.partition import groups_two_fronts, window_fronts
from oracle.problem import moving_profile, moving_profile_above


def test_two_front_groups_and_windows():
    G = groups_two_fronts(15, 3, 2)
    assert G == [(1, 3), (4, 5), (6, 7), (8, 9), (10, 11), (12, 12), (13, 15)]
    mid = len(G) // 2
    assert mid == 3
    assert window_fronts(G, 0, 2, 2) == (1, 3, None, None)
    assert window_fronts(G, 6, 2, 2) == (13, 15, None, None)
    assert window_fronts(G, 1, 2, 2) == (2, 5, 4, None)          # below the middle: padded below
    assert window_fronts(G, 5, 2, 2) == (12, 14, None, 12)       # above: padded above
    assert window_fronts(G, 3, 2, 2) == (6, 11, 8, 9)            # middle: both sides
    # every node in exactly one group
    nodes = [k for a, e in G for k in range(a, e + 1)]
    assert nodes == list(range(1, 16))


def test_moving_profile_above_is_the_mirror_image():
    """The PML padded above node e equals the one padded below node n+1-e under x -> 1-x
    (half-step position t -> 2(n+1) - t)."""
    n, p, C, om = 20, 4, 17.0, 9.0
    for e in (8, 13):
        t = np.arange(2 * e, 2 * (e + p + 1) + 1)
        up = moving_profile_above(t, e, p, n, C, om)
        down = moving_profile(2 * (n + 1) - t, n + 1 - e, p, n, C, om)
        assert np.allclose(up, down, rtol=1e-15, atol=0)
    # undamped at the last physical node, damped at the padding, sigma = 0 outside
    assert moving_profile_above(2 * 8, 8, p, n, C, om) == 1.0
    assert abs(moving_profile_above(2 * 9, 8, p, n, C, om) - 1.0) > 1e-3


def _mirror_z(v, n):
    """x3 -> 1 - x3 on vectors ordered x1 fastest (unknown (k, j, i) -> (n-1-k, j, i))."""
    return np.asarray(v).reshape(n, n, n, -1)[::-1].reshape(n ** 3, -1)


@pytest.mark.parametrize("n,b,p", [(11, 3, 3), (13, 3, 2)])
def test_two_front_sweep_commutes_with_x3_mirror(n, b, p):
    """With a medium symmetric in x3 and a symmetric two-front partition (d = 1 and n - 2b odd,
    so the middle group is the central layer), the preconditioner
    commutes with the reflection x3 -> 1 - x3: the front sweeping down from x3 = 1 and the
    middle slab's double-sided PML are the mirror images of the other side.  (The one-front
    sweep does not have this symmetry.)"""
    case = inputs.small_case(n=n, b=b, p=p, d=1)
    c = case["c"]
    c = 0.5 * (c + c[::-1])                      # symmetric in x3
    kw = dict(n=n, c=c, omega=case["omega"], b=b, C=case["C"], p=p, d=1)
    M2 = O.RecursiveSweep(O.Problem(fronts=2, **kw))
    f = inputs.random_rhs(n, 2, seed=19).reshape(2, -1).T
    lhs = M2.apply(_mirror_z(f, n))
    rhs = _mirror_z(M2.apply(f), n)
    assert _rel(lhs, rhs) < 1e-12
    M1 = O.RecursiveSweep(O.Problem(fronts=1, **kw))
    assert _rel(M1.apply(_mirror_z(f, n)), _mirror_z(M1.apply(f), n)) > 1e-6


def test_two_front_preconditioner_linear_adjoint_and_effective():
    prob = _prob(n=11, fronts=2)
    M = O.RecursiveSweep(prob)
    x, y = inputs.random_rhs(11, 2, seed=7).reshape(2, -1)
    a, bb = 0.3 - 1.1j, 2.0 + 0.5j
    assert _rel(M.apply(a * x + bb * y)[:, 0], a * M.apply(x)[:, 0] + bb * M.apply(y)[:, 0]) < 1e-13
    d1 = np.vdot(M.apply(x)[:, 0], y)
    d2 = np.vdot(x, M.apply(y, adjoint=True)[:, 0])
    assert abs(d1 - d2) <= 1e-13 * abs(d1)
    # as good an approximate inverse as the single front: GMRES converges to the direct solve
    f = inputs.random_rhs(11, 1, seed=3).reshape(-1)
    xs = spla.spsolve(M.A.tocsc(), f)
    z = M.apply(f)[:, 0]
    assert _rel(z, xs) < 0.8
    u, its, _ = O.fgmres(lambda v: M.A @ v, lambda v: M.apply(v)[:, 0], f, tol=1e-10, restart=40, maxit=80)
    assert _rel(u, xs) < 1e-8
    M1 = O.RecursiveSweep(_prob(n=11))
    _, its1, _ = O.fgmres(lambda v: M1.A @ v, lambda v: M1.apply(v)[:, 0], f, tol=1e-10, restart=40, maxit=80)
    assert its <= its1 + 3, (its, its1)


def _mirror_y(v, n):
    """x2 -> 1 - x2 on vectors ordered x1 fastest (unknown (k, j, i) -> (k, n-1-j, i))."""
    return np.asarray(v).reshape(n, n, n, -1)[:, ::-1].reshape(n ** 3, -1)


@pytest.mark.parametrize("fronts", [1, 2])
def test_two_inner_fronts_commute_with_x2_mirror(fronts):
    """Two fronts in the inner sweep (x2): with a medium symmetric in x2 and a symmetric x2
    partition, M^{-1} commutes with x2 -> 1 - x2 (the single inner front does not)."""
    n, b, p = 11, 3, 3
    case = inputs.small_case(n=n, b=b, p=p, d=1)
    c = case["c"]
    c = 0.5 * (c + c[:, ::-1])                   # symmetric in x2
    kw = dict(n=n, c=c, omega=case["omega"], b=b, C=case["C"], p=p, d=1, fronts=fronts)
    M = O.RecursiveSweep(O.Problem(fronts_inner=2, **kw))
    f = inputs.random_rhs(n, 2, seed=23).reshape(2, -1).T
    assert _rel(M.apply(_mirror_y(f, n)), _mirror_y(M.apply(f), n)) < 1e-12
    M1 = O.RecursiveSweep(O.Problem(fronts_inner=1, **kw))
    assert _rel(M1.apply(_mirror_y(f, n)), _mirror_y(M1.apply(f), n)) > 1e-6


def test_two_inner_fronts_linear_adjoint_and_effective():
    prob = _prob(n=11, fronts=2, fronts_inner=2)
    M = O.RecursiveSweep(prob)
    x, y = inputs.random_rhs(11, 2, seed=9).reshape(2, -1)
    a, bb = 1.3 + 0.2j, -0.7 + 2.0j
    assert _rel(M.apply(a * x + bb * y)[:, 0], a * M.apply(x)[:, 0] + bb * M.apply(y)[:, 0]) < 1e-13
    d1 = np.vdot(M.apply(x)[:, 0], y)
    d2 = np.vdot(x, M.apply(y, adjoint=True)[:, 0])
    assert abs(d1 - d2) <= 1e-13 * abs(d1)
    f = inputs.random_rhs(11, 1, seed=4).reshape(-1)
    xs = spla.spsolve(M.A.tocsc(), f)
    u, its, _ = O.fgmres(lambda v: M.A @ v, lambda v: M.apply(v)[:, 0], f, tol=1e-10, restart=40, maxit=80)
    assert _rel(u, xs) < 1e-8
    M1 = O.RecursiveSweep(_prob(n=11))
    _, its1, _ = O.fgmres(lambda v: M1.A @ v, lambda v: M1.apply(v)[:, 0], f, tol=1e-10, restart=40, maxit=80)
    assert its <= its1 + 3, (its, its1)


@pytest.mark.parametrize("fronts,fronts_inner", [(1, 1), (2, 2)])
def test_line_problem_depends_on_its_window_only(fronts, fronts_inner):
    """Sec. 6 (local updates): a change of c inside a box changes the line problem (g, l)
    exactly when the box meets its x3-window and its x2-window (a line spans all of x1).  This
    is the selection rule of the library's local factor update."""
    n, b, p, d = 13, 3, 3, 2
    case = inputs.small_case(n=n, b=b, p=p, d=d)
    c = case["c"]
    box = (4, 9, 6, 7, 9, 10)                   # i0, i1, j0, j1, k0, k1 (1-based)
    c2 = c.copy()
    c2[box[4] - 1:box[5], box[2] - 1:box[3], box[0] - 1:box[1]] *= 1.07
    kw = dict(n=n, omega=case["omega"], b=b, C=case["C"], p=p, d=d, fronts=fronts, fronts_inner=fronts_inner)
    P1, P2 = O.Problem(c=c, **kw), O.Problem(c=c2, **kw)
    Gz = O.groups_two_fronts(n, b, d) if fronts == 2 else O.groups(n, b, d)
    Gy = O.groups_two_fronts(n, b, d) if fronts_inner == 2 else O.groups(n, b, d)
    changed = 0
    for g in range(len(Gz)):
        zw0, zw1, _, _ = O.window_fronts(Gz, g, p, fronts)
        for l in range(len(Gy)):
            yw0, yw1, _, _ = O.window_fronts(Gy, l, p, fronts_inner)
            K1 = O.LineFactors(P1, Gz, g, Gy, l).K
            K2 = O.LineFactors(P2, Gz, g, Gy, l).K
            meets = zw0 <= box[5] and zw1 >= box[4] and yw0 <= box[3] and yw1 >= box[2]
            same = (K1 != K2).nnz == 0
            assert same != meets, (g, l, meets)
            changed += meets
    assert 0 < changed < len(Gz) * len(Gy)


def test_moving_pml_constant_changes_the_preconditioner_only():
    """C_moving enters the auxiliary problems' moving PML, not eq. (3): A is unchanged, the
    sweep changes, and C_moving = C is the default."""
    case = inputs.small_case(n=11, b=3, p=3, d=1)
    kw = dict(n=11, c=case["c"], omega=case["omega"], b=3, C=case["C"], p=3, d=1, fronts=2, fronts_inner=2)
    M0 = O.RecursiveSweep(O.Problem(**kw))
    M1 = O.RecursiveSweep(O.Problem(C_moving=case["C"], **kw))
    M2 = O.RecursiveSweep(O.Problem(C_moving=2.0 * case["C"], **kw))
    assert (M0.A != M2.A).nnz == 0
    f = inputs.random_rhs(11, 1, seed=5).reshape(-1)
    z0, z1, z2 = M0.apply(f), M1.apply(f), M2.apply(f)
    assert np.array_equal(z0, z1)
    assert _rel(z2, z0) > 1e-3
