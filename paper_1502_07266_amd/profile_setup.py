"""Driver for profiles of the setup (block LDU of every line, Algorithms 3 and 5): builds the
handle of a workload several times (each build runs the whole setup) and prints the setup
time the library measures with HIP events, with the algorithmic flop count of the block
inversions (8 B^3 real flops per block: 4 real products of B^3/2 complex multiply-adds for the
Schur updates are not counted).

    python -m paper_1502_07266_amd.profile_setup --workload c3 --prec c64 --repeat 3

Run it under `rocprofv3 --kernel-trace --stats ...` for per-kernel times, or under
`rocprofv3 --pmc ...` for matrix-core counters of the setup kernels.
"""
import argparse
import json

import torch

from . import inputs
from .binding import Helm


def window_widths(n, b, p, d, fronts):
    """Width of every group's auxiliary window along one axis (the partition of the library's
    plan): one front, the b boundary layers then groups of d padded with p below; two fronts,
    b layers at each face, groups of d between, padded below before the middle group, above
    after it, on both sides at it."""
    if fronts == 1:
        out = [b]
        k = b + 1
        while k <= n:
            out.append(min(k + d - 1, n) - k + 1 + p)
            k += d
        return out
    cut = [(1, b)]
    k = b + 1
    while k <= n - b:
        cut.append((k, min(k + d - 1, n - b)))
        k += d
    cut.append((n - b + 1, n))
    G, mid = len(cut), len(cut) // 2
    out = []
    for g, (a, e) in enumerate(cut):
        w = e - a + 1
        if 0 < g < G - 1:
            w += p * ((g <= mid) + (g >= mid))
        out.append(w)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="c64", choices=["c64", "c128"])
    ap.add_argument("--repeat", type=int, default=3)
    ap.add_argument("--fronts", type=int, default=2, choices=[1, 2])
    ap.add_argument("--fronts-inner", type=int, default=2, choices=[1, 2])
    args = ap.parse_args()
    wl = inputs.workload(args.workload)
    c = torch.from_numpy(wl["c"]).to("cuda:0")
    ms = []
    for _ in range(args.repeat):
        H = Helm(c, wl["omega"], wl["b"], wl["C"], wl["p"], wl["d"], prec=args.prec, fronts=args.fronts,
                 fronts_inner=args.fronts_inner, C_moving=wl.get("C_moving", 0.0))
        torch.cuda.synchronize()
        ms.append(H.stats()["setup_ms"])
        H.close()
    n = wl["n"]
    wz = window_widths(n, wl["b"], wl["p"], wl["d"], args.fronts)
    wy = window_widths(n, wl["b"], wl["p"], wl["d"], args.fronts_inner)
    flops = 8.0 * n * sum(float(a * b_) ** 3 for a in wz for b_ in wy)
    print(json.dumps({"workload": args.workload, "prec": args.prec, "setup_ms": ms,
                      "inversion_flops": flops,
                      "inversion_tflops": flops / (min(ms) * 1e-3) / 1e12}), flush=True)


if __name__ == "__main__":
    main()
