"""Driver for hardware-counter runs of the sweep: one plain copy of a known size, then one
batched sweep (helm_apply: one cooperative launch of the sweep kernel) of a workload, with a
fixed launch shape (no tuning runs in between).

    python -m paper_1502_07266_amd.profile_sweep --workload c3 --prec c64 --copy-mib 1024 --variant 46
        [--line-solver nd]

Run it under `rocprofv3 --pmc FETCH_SIZE ...` and again under `--pmc WRITE_SIZE ...`: the
copy kernel reads and writes exactly copy-mib MiB, which calibrates what the counters report
per byte, and the sweep dispatch gives the sweep's memory traffic beyond L2.  Prints the
device times of both (HIP events) and the sweep's algorithmic bytes.
"""
import argparse
import json
import os
import time

import torch

from . import inputs
from .binding import Helm


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="c3")
    ap.add_argument("--prec", default="c64", choices=["c64", "c128"])
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--rhs", type=int, default=0, help="right-hand sides (0: all of the workload)")
    ap.add_argument("--fronts", type=int, default=2, choices=[1, 2])
    ap.add_argument("--fronts-inner", type=int, default=2, choices=[1, 2])
    ap.add_argument("--variant", type=int, default=-1, help="launch shape (-1: the default one)")
    ap.add_argument("--line-solver", default="ldu", choices=["ldu", "nd"],
                    help="line solves by the block LDU chains or by nested dissection (its factors are "
                         "computed before the measured sweep)")
    args = ap.parse_args()
    os.environ["HELM_AUTOTUNE"] = "0"

    wl = inputs.workload(args.workload)
    n = wl["n"]
    nodes = wl["nodes"] if args.rhs <= 0 else wl["nodes"][:args.rhs]
    R = len(nodes)
    dev = torch.device("cuda:0")

    nbytes = args.copy_mib << 20
    src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1)
    print(f"[profile] copy {args.copy_mib} MiB: {copy_ms:.3f} ms", flush=True)
    del src, dst

    c = torch.from_numpy(wl["c"]).to(dev)
    F = torch.from_numpy(inputs.sources(n, nodes)).to(dev)
    H = Helm(c, wl["omega"], wl["b"], wl["C"], wl["p"], wl["d"], prec=args.prec, fronts=args.fronts,
             fronts_inner=args.fronts_inner, C_moving=wl.get("C_moving", 0.0))
    H.set_launch(args.variant)
    if args.line_solver == "nd":
        H.set_line_solver("nd")
    H.reset_stats()
    t0 = time.perf_counter()
    H.apply(F)
    torch.cuda.synchronize()
    st = H.stats()
    kbytes = st["kernel_bytes"] / max(st["kernel_launches"], 1)
    if args.line_solver == "nd":
        # the library counts the block LDU factors (n blocks per line visit); nested dissection
        # reads 3 n - 2 popcount(n) blocks of its own per line visit
        vec = 32.0 * n ** 3 * R
        kbytes = (kbytes - vec) * (3 * n - 2 * bin(n).count("1")) / n + vec
    print(f"[profile] apply {args.prec} R={R}: {st['apply_ms']:.1f} ms "
          f"(host {1e3 * (time.perf_counter() - t0):.1f} ms)", flush=True)
    print(json.dumps({"workload": args.workload, "prec": args.prec, "rhs": R, "fronts": args.fronts,
                      "fronts_inner": args.fronts_inner, "b": wl["b"], "p": wl["p"], "d": wl["d"],
                      "C_moving": wl.get("C_moving", 0.0), "line_solver": args.line_solver,
                      "copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copy_ms": copy_ms,
                      "apply_ms": st["apply_ms"],
                      "apply_algorithmic_bytes": st["apply_bytes_per_rhs"] * R,
                      "kernel_launches": st["kernel_launches"], "kernel_ms": st["kernel_ms"],
                      "shape": H.sweep_shape(R)[1],
                      "kernel_algorithmic_bytes_per_launch": kbytes}),
          flush=True)
    H.close()


if __name__ == "__main__":
    main()
