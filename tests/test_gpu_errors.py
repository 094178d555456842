"""Error paths of the library on the GPU, forced from the host with valid kernels: a solve whose
planned Krylov workspace exceeds the device's memory is refused with HELM_ENOMEM before any of
it is allocated (the bytes are planned from the batch, the restart length and the iteration
cap), and a setup whose Schur complements are not finite (omega^2 overflows kappa) reports
HELM_ESINGULAR with the line, and the handle is not created."""
import numpy as np
import pytest
import torch

from paper_1502_07266_amd import inputs
from paper_1502_07266_amd.binding import HELM_ENOMEM, HELM_ESINGULAR, Helm, HelmError, pool_stats

pytestmark = pytest.mark.gpu


def _small(prec, omega=None):
    sc = inputs.small_case(n=15, b=3, p=3, d=1)
    c = torch.from_numpy(sc["c"]).cuda()
    return Helm(c, sc["omega"] if omega is None else omega, 3, sc["C"], 3, 1, prec=prec)


def test_solve_beyond_device_memory_is_enomem_before_allocating():
    H = _small("c64")
    H.set_launch(H.sweep_shape(1)[0])   # a fixed launch shape: no tuning sweeps before the solve
    n = H.n
    total = torch.cuda.mem_get_info()[1]
    R = int(total // H.workspace_bytes(1, 200, 200)["solve"]) + 2
    while H.workspace_bytes(R, 200, 200)["solve"] <= total:   # the planned bytes are not linear in R
        R = R + R // 16 + 1
    f = torch.zeros((R, n, n, n), dtype=torch.complex128, device="cuda")
    f[:, n // 2, n // 2, n // 2] = 1.0
    live_before = pool_stats()[1]
    with pytest.raises(HelmError) as e:
        H.solve(f, tol=1e-6, restart=200, maxit=200)
    assert e.value.code == HELM_ENOMEM
    assert "bytes" in str(e.value)
    assert pool_stats()[1] == live_before      # nothing of the workspace was taken
    # the handle still solves a batch that fits
    u, its, rel, rc = H.solve(f[:2], tol=1e-6, restart=20, maxit=40)
    assert rc == 0 and float(rel.max()) <= 1e-6
    H.close()


@pytest.mark.parametrize("prec", ["c64", "c128"])
def test_setup_with_non_finite_blocks_is_esingular(prec):
    with pytest.raises(HelmError) as e:
        _small(prec, omega=1e160)           # omega^2 / c^2 is infinite in double precision
    assert e.value.code == HELM_ESINGULAR
    assert "line" in str(e.value)
    # the library keeps working afterwards
    H = _small(prec)
    x = torch.from_numpy(inputs.random_rhs(H.n, 1, seed=3)).cuda()
    z = H.apply(x)
    assert bool(torch.isfinite(torch.view_as_real(z)).all())
    H.close()
