"""Velocity gradient of the receiver misfit at full size, against central differences.

    python -m paper_1502_07266_amd.gradient_check [--cells 20] [--prec c64] [--tol 1e-12]

Workload: 63^3, two-layer medium with a 5 % seeded perturbation, omega = 2 pi 8, 8 sources
on x3 = 0.1, receivers on every node of the x3-layer nearest 0.9, data synthesised from the
unperturbed medium.  The gradient dJ/dc comes from one forward and one adjoint solve
(helm_solve, helm_misfit, helm_grad_c through torch.autograd); each of the seeded non-PML
cells is checked against (J(c + e) - J(c - e)) / (2 e) with e = 1e-4, every J from a solve
to relative residual `tol` (FGMRES in FP64 around the complex64 or complex128 sweep).  The
preconditioner's configuration (--p, --d, fronts) changes only the speed of those solves;
the default d = 3, p = 4 with two fronts in both axes is the fastest at this size.  Prints
one JSON line per cell and a summary line.
"""
import argparse
import json
import sys
import time

import numpy as np


def run(cells=20, prec="c64", tol=1e-12, p=4, d=3, fronts=2, fronts_inner=2, log=None):
    import torch
    from . import inputs
    from .autograd import misfit
    from .binding import Helm
    wl = inputs.workload("c4")
    n, plane = wl["n"], wl["plane_k"]
    dev = torch.device("cuda:0")
    F = torch.from_numpy(inputs.sources(n, wl["nodes"])).to(dev)
    kw = dict(omega=wl["omega"], b=wl["b"], C=wl["C"], p=p, slab_layers=d, prec=prec, tol=tol,
              restart=wl["restart"], maxit=400, fronts=fronts, fronts_inner=fronts_inner)
    # data from the unperturbed medium
    H0 = Helm(torch.from_numpy(wl["c0"]).to(dev), wl["omega"], wl["b"], wl["C"], p, d, prec=prec,
              fronts=fronts, fronts_inner=fronts_inner)
    u0, its0, _, _ = H0.solve(F, tol=tol, restart=wl["restart"], maxit=400)
    H0.close()
    d_obs = u0[:, plane - 1].contiguous()
    del u0
    c0 = torch.from_numpy(wl["c"]).to(dev)
    c = c0.clone().requires_grad_(True)
    t0 = time.perf_counter()
    J = misfit(c, F, d_obs, plane, **kw)
    J.backward()
    torch.cuda.synchronize()
    t_grad = time.perf_counter() - t0
    g = c.grad.cpu().numpy()
    eps = wl["fd_step"]
    gscale = float(np.abs(g).max())
    rows = []
    for (i, j, k) in wl["fd_cells"][:cells]:
        cp, cm = c0.clone(), c0.clone()
        cp[k - 1, j - 1, i - 1] += eps
        cm[k - 1, j - 1, i - 1] -= eps
        with torch.no_grad():
            Jp = misfit(cp, F, d_obs, plane, **kw).item()
            Jm = misfit(cm, F, d_obs, plane, **kw).item()
        fd = (Jp - Jm) / (2 * eps)
        ga = float(g[k - 1, j - 1, i - 1])
        row = {"cell": [int(i), int(j), int(k)], "adjoint": ga, "central_difference": fd,
               "rel_err": abs(fd - ga) / max(abs(fd), 1e-3 * gscale)}
        rows.append(row)
        if log:
            log(json.dumps(row))
    return {"J": float(J.item()), "gradient_s": round(t_grad, 3), "cells": len(rows),
            "max_rel_err": max(r["rel_err"] for r in rows), "grad_max_abs": gscale,
            "prec": prec, "tol": tol, "p": p, "d": d, "fronts": fronts, "fronts_inner": fronts_inner}, rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cells", type=int, default=20)
    ap.add_argument("--prec", default="c64", choices=["c64", "c128"])
    ap.add_argument("--tol", type=float, default=1e-12)
    ap.add_argument("--p", type=int, default=4)
    ap.add_argument("--d", type=int, default=3)
    ap.add_argument("--fronts", type=int, default=2)
    ap.add_argument("--fronts-inner", type=int, default=2)
    args = ap.parse_args()
    summary, _ = run(args.cells, args.prec, args.tol, args.p, args.d, args.fronts, args.fronts_inner,
                     log=lambda s: print(s, flush=True))
    print(json.dumps(summary), flush=True)
    return 0 if summary["max_rel_err"] <= 1e-4 else 1


if __name__ == "__main__":
    sys.exit(main())
