"""The experiments of Sec. 5 with the paper's settings, on one GPU.

    python -m paper_1502_07266_amd.paper_tables [--sizes 63,127] [--media a,b,c,a-,b-]
                                                [--forces a,b] [--prec c64]

Settings as in Sec. 5: q = 8 points per wavelength (omega / 2 pi = (n + 1) / 8), boundary
PML 9h, auxiliary (moving) PML 5h, 4 layers per auxiliary problem, two fronts in the outer
loop, GMRES(40) to relative residual 1e-3; the inner loop runs one front (with two, the
middle-middle line would have 14 x 14 = 196 unknowns per block, beyond the sweep's one-chain
limit of 128), and the boundary PML constant is C = 30 b as in the other workloads.  At
255^3 (52.8 GB of complex64 factors) a solve of one right-hand side takes about a minute.
Media (Sec. 5; synthetic stand-ins, the paper gives figures only):
(a) Gaussian lens and (b) vertical Gaussian waveguide with c = 1 + 0.4 exp(-r^2 / 0.02), so
that q = 8 holds everywhere (c >= 1); (a-) and (b-) the same with c = 1 - 0.4 exp(...), whose
slow centre has only 4.8 points per wavelength; (c) random field in [1, 2].  Forces: (a) a Gaussian point source at
(1/2, 1/2, 1/4) (standard deviation 2h), (b) a Gaussian wave packet at (1/2, 1/4, 1/4)
travelling along (0, 1, 1)/sqrt(2) with the wavelength of c = 1 (envelope standard deviation
one wavelength).  Prints one JSON line per solve and, at the end, a table of iteration counts
beside the paper's (Tables 1-3, column N_iter R).
"""
import argparse
import json
import math
import sys
import time

import numpy as np

from . import inputs

# N_iter of the recursive method in the paper: Table 1 (lens), Table 2 (waveguide), Table 3
# (random medium); keys (medium, n, force)
PAPER_ITERS = {
    ("a", 63, "a"): 4, ("a", 63, "b"): 4, ("a", 127, "a"): 4, ("a", 127, "b"): 4,
    ("a", 255, "a"): 5, ("a", 255, "b"): 5,
    ("b", 63, "a"): 4, ("b", 63, "b"): 5, ("b", 127, "a"): 5, ("b", 127, "b"): 5,
    ("b", 255, "a"): 6, ("b", 255, "b"): 5,
    ("c", 63, "a"): 4, ("c", 63, "b"): 4, ("c", 127, "a"): 4, ("c", 127, "b"): 5,
    ("c", 255, "a"): 5, ("c", 255, "b"): 6,
}


def medium(name, n):
    if name in ("a", "a-"):
        return inputs.medium_lens(n, 0.4 if name == "a" else -0.4)
    if name in ("b", "b-"):
        return inputs.medium_waveguide(n, 0.4 if name == "b" else -0.4)
    return inputs.medium_grf(n, 0.1, 1.0, 2.0)


def force(name, n, omega):
    h = inputs.grid_h(n)
    if name == "a":
        return inputs.force_gaussian(n, (0.5, 0.5, 0.25), 2.0 * h)
    lam = 2.0 * math.pi / omega
    d = (0.0, 1.0 / math.sqrt(2.0), 1.0 / math.sqrt(2.0))
    return inputs.force_wave_packet(n, (0.5, 0.25, 0.25), d, omega, lam)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--sizes", default="63,127")
    ap.add_argument("--media", default="a,b,c,a-,b-")
    ap.add_argument("--forces", default="a,b")
    ap.add_argument("--prec", default="c64", choices=["c64", "c128"])
    ap.add_argument("--b", type=int, default=9)
    ap.add_argument("--p", type=int, default=5)
    ap.add_argument("--d", type=int, default=4)
    ap.add_argument("--fronts", type=int, default=2)
    ap.add_argument("--fronts-inner", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--restart", type=int, default=40)
    ap.add_argument("--maxit", type=int, default=60)
    args = ap.parse_args()

    import torch
    from .binding import Helm
    rows = []
    for n in [int(v) for v in args.sizes.split(",")]:
        omega = 2.0 * math.pi * (n + 1) / 8.0
        for med in args.media.split(","):
            c = torch.from_numpy(medium(med, n)).cuda()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            H = Helm(c, omega, args.b, 30.0 * args.b, args.p, args.d, prec=args.prec,
                     fronts=args.fronts, fronts_inner=args.fronts_inner)
            torch.cuda.synchronize()
            t_setup = time.perf_counter() - t0
            for frc in args.forces.split(","):
                f = torch.from_numpy(force(frc, n, omega)).cuda()
                print(f"[tables] n={n} medium ({med}) force ({frc})", file=sys.stderr, flush=True)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                u, its, rel, rc = H.solve(f, tol=args.tol, restart=args.restart, maxit=args.maxit)
                torch.cuda.synchronize()
                t_solve = time.perf_counter() - t1
                row = {"n": n, "omega_over_2pi": (n + 1) / 8.0, "medium": med, "force": frc,
                       "iters": int(its[0]), "relres": float(rel[0]), "status": rc,
                       "setup_s": round(t_setup, 3), "solve_s": round(t_solve, 3),
                       "paper_iters": PAPER_ITERS.get((med.rstrip("-"), n, frc))}
                rows.append(row)
                print(json.dumps(row), flush=True)
                del u, f
            H.close()
            del c
    print("| medium | n | force | iterations | paper (R) | setup s | solve s |")
    print("|---|---|---|---|---|---|---|")
    for r in rows:
        print(f"| ({r['medium']}) | {r['n']}^3 | ({r['force']}) | {r['iters']} | {r['paper_iters']} | "
              f"{r['setup_s']} | {r['solve_s']} |")


if __name__ == "__main__":
    main()
