"""GPU parity of the nested-dissection line solver (helm_set_line_solver, Sec. 6: 1D nested
dissection of each line, done as block cyclic reduction in x1) against the oracle.

The nested-dissection solve is Gaussian elimination of the same line matrices in another
order, so the preconditioner is the one the block LDU chains apply, up to rounding: the
sweeps are compared with the oracle's Algorithm 6 (block LDU line solves) at the complex64
bound of the chain path (1.2e-5, observed errors about 1e-6), line solves with the oracle's
sparse line solve, solves with a sparse direct solve of eq. (3).  It needs n = 2^k - 1.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from paper_1502_07266_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CASES = {
    "tiny3": dict(n=3, b=1, p=1, d=1),
    "tiny3_2f2i": dict(n=3, b=1, p=1, d=1, fronts=2, fronts_inner=2),
    "n7_2f2i": dict(n=7, b=2, p=1, d=1, fronts=2, fronts_inner=2),
    "b4p4": dict(n=15, b=4, p=4, d=1),
    "b4p4_2f": dict(n=15, b=4, p=4, d=1, fronts=2),
    "b4p4_2f2i": dict(n=15, b=4, p=4, d=1, fronts=2, fronts_inner=2),
    "b4p4_1f2i": dict(n=15, b=4, p=4, d=1, fronts=1, fronts_inner=2),
    "b4p4_2f2i_cm": dict(n=15, b=4, p=4, d=1, fronts=2, fronts_inner=2, C_moving_scale=2.0),
    # 31 blocks per line (five levels); ragged last groups; blocks of 9 x 9 = 81 > 64
    # unknowns (two rows per lane in the products)
    "n31_2f2i": dict(n=31, b=4, p=3, d=3, fronts=2, fronts_inner=2),
    "n31_wide": dict(n=31, b=3, p=3, d=6),
}
_cache = {}
APPLY_TOL_C64 = 1.2e-5


def case(name):
    if name not in _cache:
        cfg = CASES[name]
        sc = inputs.small_case(n=cfg["n"], b=cfg["b"], p=cfg["p"], d=cfg["d"])
        prob = O.Problem(n=cfg["n"], c=sc["c"], omega=sc["omega"], b=cfg["b"], C=sc["C"], p=cfg["p"], d=cfg["d"],
                         fronts=cfg.get("fronts", 1), fronts_inner=cfg.get("fronts_inner", 1),
                         C_moving=cfg.get("C_moving_scale", 0.0) * sc["C"])
        _cache[name] = (sc, prob, O.RecursiveSweep(prob))
    return _cache[name]


def helm(name, solver="nd", c=None):
    from paper_1502_07266_amd.binding import Helm
    sc, prob, _ = case(name)
    cc = torch.from_numpy(sc["c"] if c is None else c).cuda()
    H = Helm(cc, sc["omega"], prob.b, prob.C, prob.p, prob.d, prec="c64", fronts=prob.fronts,
             fronts_inner=prob.fronts_inner, C_moving=prob.C_moving)
    H.set_line_solver(solver)
    return H


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


def to_gpu(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


@pytest.mark.parametrize("name", list(CASES))
def test_nd_apply(name):
    sc, prob, M = case(name)
    n = prob.n
    x = inputs.random_rhs(n, 3, seed=5)
    print(f"== nd apply {name}", flush=True)
    H = helm(name)
    z = H.apply(to_gpu(x)).cpu().numpy()
    ref = M.apply(x.reshape(3, -1).T).T.reshape(x.shape)
    err = max(rel(z[q], ref[q]) for q in range(3))
    H.set_line_solver("ldu")
    zc = H.apply(to_gpu(x)).cpu().numpy()
    print(f"nd apply {name}: vs oracle {err:.2e}, vs block LDU chains {rel(z, zc):.2e}")
    assert err <= APPLY_TOL_C64
    assert rel(z, zc) <= 2 * APPLY_TOL_C64
    H.close()


@pytest.mark.parametrize("name", ["tiny3", "n7_2f2i", "b4p4_2f2i", "n31_2f2i", "n31_wide"])
def test_nd_line_solve(name):
    """Line solves on random right-hand sides against the oracle's sparse line solve.
    Complex64 rounding is amplified by the line's conditioning, and cyclic reduction more than
    the chains: every level multiplies by inverses of reduced blocks (observed: up to 1.0e-5,
    14 x the chains' 7e-7 on the same lines).  Bound 5e-5; the sweep-level bound is the
    chains' (test_nd_apply)."""
    sc, prob, M = case(name)
    print(f"== nd line solve {name}", flush=True)
    H = helm(name)
    rng = np.random.default_rng(3)
    Gz, Gy = len(M.Gz), len(M.Gy)
    worst_nd = worst_ldu = 0.0
    for (g, l) in sorted({(0, 0), (Gz - 1, Gy - 1), (Gz // 2, 0), (0, Gy // 2), (Gz // 2, Gy // 2), (1 % Gz, 2 % Gy)}):
        ln = M.slabs[g].lines[l]
        Nl = ln.K.shape[0]
        r = rng.standard_normal((2, Nl)) + 1j * rng.standard_normal((2, Nl))
        ref = ln.solve(r.T).T
        rg = to_gpu(r.reshape(2, ln.Wz, ln.Wy, prob.n))
        H.set_line_solver("nd")
        worst_nd = max(worst_nd, rel(H.line_solve(g, l, rg).cpu().numpy().reshape(2, -1), ref))
        H.set_line_solver("ldu")
        worst_ldu = max(worst_ldu, rel(H.line_solve(g, l, rg).cpu().numpy().reshape(2, -1), ref))
    print(f"nd line solve {name}: worst {worst_nd:.2e} (block LDU chains {worst_ldu:.2e})")
    assert worst_nd <= 5e-5
    H.close()


@pytest.mark.parametrize("name", ["tiny3_2f2i", "b4p4", "b4p4_2f2i", "n31_2f2i", "n31_wide"])
def test_nd_solve(name):
    sc, prob, M = case(name)
    n = prob.n
    f = inputs.random_rhs(n, 2, seed=13)
    print(f"== nd solve {name}", flush=True)
    H = helm(name)
    u, its, relres, rc = H.solve(to_gpu(f), tol=1e-8, restart=30, maxit=200)
    u = u.cpu().numpy()
    ref = spla.spsolve(M.A.tocsc(), f.reshape(2, -1).T).T.reshape(f.shape)
    errs = [rel(u[q], ref[q]) for q in range(2)]
    print(f"nd solve {name}: its {its} relres {relres} err {max(errs):.2e}")
    assert rc == 0 and np.all(relres <= 1e-8)
    assert max(errs) <= 1e-6
    for q in range(2):
        r = f[q].ravel() - M.A @ u[q].ravel()
        assert np.linalg.norm(r) <= 1.01e-8 * np.linalg.norm(f[q])
    H.close()


def test_nd_placements_give_the_same_sweep():
    """The workgroup placement moves members between XCDs, not arithmetic: bit-identical."""
    sc, prob, M = case("b4p4_2f2i")
    H = helm("b4p4_2f2i")
    x = to_gpu(inputs.random_rhs(prob.n, 5, seed=7))
    v = H.sweep_shape(5)[0] // 4
    outs = []
    for m in range(3):
        H.set_launch(4 * v + m)
        outs.append(H.apply(x))
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    H.close()


def test_nd_update_medium_refactors():
    """helm_update_medium refactors the nested-dissection factors as well: the sweep equals
    a fresh handle's on the new medium, bit for bit."""
    from paper_1502_07266_amd.binding import Helm
    sc, prob, M = case("b4p4_2f2i")
    n = prob.n
    box = (3, n - 4, 5, 7, n - 6, n - 5)
    c2 = sc["c"].copy()
    c2[box[4] - 1:box[5], box[2] - 1:box[3], box[0] - 1:box[1]] *= 1.07
    H = helm("b4p4_2f2i")
    H.update_medium(torch.from_numpy(c2).cuda(), box)
    H2 = helm("b4p4_2f2i", c=c2)
    x = to_gpu(inputs.random_rhs(n, 2, seed=17))
    assert torch.equal(H.apply(x), H2.apply(x))
    H.close()
    H2.close()


def test_nd_unsupported_plans_are_rejected():
    from paper_1502_07266_amd.binding import HELM_EINVAL, Helm, HelmError
    sc = inputs.small_case(n=16, b=3, p=2, d=2)
    H = Helm(torch.from_numpy(sc["c"]).cuda(), sc["omega"], 3, sc["C"], 2, 2, prec="c64")
    with pytest.raises(HelmError) as e:
        H.set_line_solver("nd")          # n + 1 is not a power of two
    assert e.value.code == HELM_EINVAL
    H.close()
    sc = inputs.small_case(n=15, b=4, p=4, d=1)
    H = Helm(torch.from_numpy(sc["c"]).cuda(), sc["omega"], 4, sc["C"], 4, 1, prec="c128")
    with pytest.raises(HelmError) as e:
        H.set_line_solver("nd")          # complex128 factors
    assert e.value.code == HELM_EINVAL
    H.close()


def test_nd_at_the_benchmarked_127cubed_configuration():
    """127^3, 32 sources, d = 5, p = 2, two fronts in x3 and x2: the nested-dissection sweep
    equals the block LDU chains' to the complex64 bound of the full-size apply (3e-5,
    observed 7.3e-6), and a solve with it reaches the tolerance in the chains' iterations
    (within one) with its true residual recomputed in FP64 by the library's matvec."""
    from paper_1502_07266_amd.binding import Helm
    wl = inputs.workload("c3")
    n = wl["n"]
    print("== nd at 127^3", flush=True)
    c = torch.from_numpy(wl["c"]).cuda()
    F = torch.from_numpy(inputs.sources(n, wl["nodes"])).cuda()
    H = Helm(c, wl["omega"], wl["b"], wl["C"], wl["p"], wl["d"], prec="c64", fronts=2, fronts_inner=2,
             C_moving=wl["C_moving"])
    H.set_launch(H.sweep_shape(32)[0])
    z_ldu = H.apply(F)
    u_ldu, its_ldu, rel_ldu, rc_ldu = H.solve(F, tol=wl["tol"], restart=wl["restart"], maxit=100)
    H.set_line_solver("nd")
    z_nd = H.apply(F)
    err = float(torch.linalg.vector_norm(z_nd - z_ldu) / torch.linalg.vector_norm(z_ldu))
    u_nd, its_nd, rel_nd, rc_nd = H.solve(F, tol=wl["tol"], restart=wl["restart"], maxit=100)
    r = F - H.matvec(u_nd)
    true_rel = (torch.linalg.vector_norm(r.reshape(32, -1), dim=1) /
                torch.linalg.vector_norm(F.reshape(32, -1), dim=1)).cpu().numpy()
    print(f"nd at 127^3: apply vs chains {err:.2e}; iterations {its_nd.tolist()} "
          f"(chains {its_ldu.tolist()}); true residual max {true_rel.max():.2e}")
    assert err <= 3e-5
    assert rc_nd == 0 and rc_ldu == 0
    assert np.all(np.abs(np.asarray(its_nd) - np.asarray(its_ldu)) <= 1)
    assert float(true_rel.max()) <= 1.01 * wl["tol"]
    H.close()


def test_nd_static_apply_equals_apply():
    """The allocation-free entry point runs the same nested-dissection kernel: helm_apply_static
    equals helm_apply bit for bit, twice in a row (the second call with fewer right-hand sides),
    with neither the library's pool nor torch's allocator growing."""
    import ctypes
    from paper_1502_07266_amd.binding import lib, pool_stats
    sc, prob, M = case("b4p4_2f2i")
    H = helm("b4p4_2f2i")
    for R in (5, 2):
        x = to_gpu(inputs.random_rhs(prob.n, R, seed=40 + R))
        ref = H.apply(x)
        z = torch.empty_like(x)
        torch.cuda.synchronize()
        pool, mem = pool_stats(), torch.cuda.memory_allocated()
        rc = lib().helm_apply_static(H.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(z.data_ptr()), R, 0,
                                     ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
        assert rc == 0
        assert pool_stats() == pool and torch.cuda.memory_allocated() == mem
        assert torch.equal(z, ref)
    H.close()
