"""helm_apply_static, the entry point that allocates nothing: through the C ABI, two calls in a
row (the second with fewer right-hand sides) against helm_apply on the same handle, bit for
bit (the same kernels and launch shape), with neither the library's pool nor torch's
allocator growing during the calls."""
import ctypes

import numpy as np
import pytest

from paper_1502_07266_amd import inputs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _static_apply(H, x, z, adjoint):
    from paper_1502_07266_amd.binding import lib
    torch.cuda.synchronize()
    rc = lib().helm_apply_static(H.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(z.data_ptr()),
                                 x.shape[0], int(adjoint), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    return rc, z


def _check(H, n, Rs, seed, adjoint=False):
    from paper_1502_07266_amd.binding import pool_stats
    for R in Rs:
        x = torch.from_numpy(inputs.random_rhs(n, R, seed=seed + R)).cuda()
        ref = H.apply(x, adjoint=adjoint)
        z = torch.empty_like(x)
        torch.cuda.synchronize()
        pool, mem = pool_stats(), torch.cuda.memory_allocated()
        rc, z = _static_apply(H, x, z, adjoint)
        assert rc == 0
        assert pool_stats() == pool, "the library's pool changed during helm_apply_static"
        assert torch.cuda.memory_allocated() == mem
        diff = float((z - ref).norm() / ref.norm())
        print(f"static apply n={n} R={R} adjoint={adjoint}: rel diff to helm_apply {diff:.1e}")
        assert torch.equal(z, ref), diff


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_static_apply_small_two_fronts(prec):
    from paper_1502_07266_amd.binding import Helm
    sc = inputs.small_case(n=15, b=4, p=4)
    c = torch.from_numpy(sc["c"]).cuda()
    H = Helm(c, sc["omega"], 4, sc["C"], 4, 1, prec=prec, fronts=2, fronts_inner=2)
    _check(H, 15, (12, 3), seed=60)
    _check(H, 15, (5, 2), seed=70, adjoint=True)
    H.close()


def test_static_apply_127_cubed_batch():
    """The benchmarked 127^3 configuration: 32 right-hand sides, then 5."""
    from paper_1502_07266_amd.binding import Helm
    wl = inputs.workload("c3")
    H = Helm(torch.from_numpy(wl["c"]).cuda(), wl["omega"], wl["b"], wl["C"], wl["p"], wl["d"], prec="c64",
             C_moving=wl["C_moving"], fronts=2, fronts_inner=2)
    _check(H, wl["n"], (32, 5), seed=80)
    H.close()
