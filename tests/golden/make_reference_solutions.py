"""Writes the oracle's reference solutions of the full-size workloads for the GPU parity tests.

Calls only ``oracle`` (and the seeded input generators of ``paper_1502_07266_amd.inputs``,
which hold none of the method's arithmetic).  Each reference is A u = f (eq. (3)) solved by
the oracle's flexible GMRES (Sec. 5 solves with GMRES) to relative residual 1e-10, with the
oracle's recursive sweep (Algorithm 6 with Algorithm 4, Sec. 4.2) of the benchmarked
configuration as the preconditioner; the solution of A u = f does not depend on that choice.

Stored per workload (``<name>_reference.npz``):
  nodes      the right-hand sides' source nodes (1-based (i, j, k)),
  stride     the subsampling step s: ``sub`` holds u[:, ::s, ::s, ::s] (indices [k, j, i]),
  sub        the subsampled solutions (complex128),
  norms      ||u||_2 of each full solution,
  relres     the oracle's final true relative residuals,
  iters      FGMRES iterations.
The 127^3 reference takes about 10 minutes on 8 cores: run it when the workload or the
oracle changes,

    python tests/golden/make_reference_solutions.py c3 c2
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O                                   # noqa: E402
from paper_1502_07266_amd import inputs              # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

# (workload, sources taken, subsampling stride, fronts, fronts_inner)
SPECS = {
    "c3": (2, 4, 2, 2),   # the batched 127^3 workload: its first two of 32 sources
    "c2": (1, 2, 1, 1),   # 63^3 lens, its single source
}


def make(name):
    count, stride, fronts, fronts_inner = SPECS[name]
    wl = inputs.workload(name)
    n = wl["n"]
    nodes = wl["nodes"][:count]
    t0 = time.time()
    prob = O.Problem(n=n, c=wl["c"], omega=wl["omega"], b=wl["b"], C=wl["C"], p=wl["p"], d=wl["d"],
                     C_moving=wl.get("C_moving", 0.0), fronts=fronts, fronts_inner=fronts_inner)
    M = O.RecursiveSweep(prob)
    print(f"{name}: oracle setup {time.time() - t0:.1f} s", flush=True)
    F = inputs.sources(n, nodes)
    subs, norms, rels, its = [], [], [], []
    for s in range(count):
        t1 = time.time()
        f = F[s].ravel()
        u, it, hist = O.fgmres(lambda x: M.A @ x, lambda r: M.apply(r), f, tol=1e-10, restart=50,
                               maxit=200)
        res = float(np.linalg.norm(f - M.A @ u) / np.linalg.norm(f))
        print(f"{name} source {s}: {it} iterations, relres {res:.2e}, {time.time() - t1:.1f} s", flush=True)
        U = u.reshape(n, n, n)
        subs.append(U[::stride, ::stride, ::stride])
        norms.append(float(np.linalg.norm(u)))
        rels.append(res)
        its.append(it)
    out = os.path.join(HERE, f"{name}_reference.npz")
    np.savez_compressed(out, nodes=np.array(nodes, dtype=np.int64), stride=np.int64(stride),
                        sub=np.stack(subs), norms=np.array(norms), relres=np.array(rels),
                        iters=np.array(its, dtype=np.int64))
    print(f"wrote {out}", flush=True)


if __name__ == "__main__":
    for name in sys.argv[1:] or list(SPECS):
        make(name)
