"""HBM traffic of one sweep kernel from two rocprofv3 counter runs of profile_sweep.

    python -m paper_1502_07266_amd.profile_traffic \\
        --fetch <dir>/fetch/run_counter_collection.csv --write <dir>/write/run_counter_collection.csv \\
        --apply-json <file with profile_sweep's JSON line> --kernel "8, 5, 8, false, 2>" --out <json>

Each CSV holds one row per dispatch and counter.  The plain copy of known size that
profile_sweep runs first (the largest __amd_rocclr_copyBuffer dispatch) calibrates each
counter: scale = bytes the copy reads (or writes) / what the counter reports for it.  The
kernel's dispatches (those whose name contains --kernel) are averaged and scaled, giving HBM
bytes per launch.  The kernel's time per launch and its algorithmic bytes per launch come from
profile_sweep's own HIP-event measurement of the same run.
"""
import argparse
import csv
import hashlib
import json
import os


def per_dispatch(path, counter):
    vals = {}
    with open(path) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] != counter:
                continue
            key = (int(r["Dispatch_Id"]), r["Kernel_Name"])
            vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return vals


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--apply-json", required=True)
    ap.add_argument("--kernel", required=True, help="substring naming the kernel instantiation")
    ap.add_argument("--out", required=True)
    args = ap.parse_args()

    with open(args.apply_json) as fh:
        run = json.loads([ln for ln in fh if ln.startswith("{")][-1])
    copy_bytes = run["copy_bytes_read"]

    out = {"workload": run["workload"], "rhs": run["rhs"], "fronts": run["fronts"],
           "fronts_inner": run.get("fronts_inner", 1), "b": run.get("b"), "p": run.get("p"),
           "d": run.get("d"), "C_moving": run.get("C_moving", 0.0), "copy_bytes": copy_bytes}
    hbm = 0.0
    for counter, path, moved in (("FETCH_SIZE", args.fetch, copy_bytes),
                                 ("WRITE_SIZE", args.write, run["copy_bytes_written"])):
        vals = per_dispatch(path, counter)
        copy_kib = max(v for (d, name), v in vals.items() if "copyBuffer" in name)
        kern = [v for (d, name), v in vals.items() if args.kernel in name and "k_sweep" in name]
        if not kern:
            raise SystemExit(f"no dispatch of a kernel matching {args.kernel!r} in {path}")
        names = {name for (d, name), v in vals.items() if args.kernel in name and "k_sweep" in name}
        out["kernel"] = sorted(names)[0]
        scale = moved / (copy_kib * 1024.0)
        avg_kib = sum(kern) / len(kern)
        tag = counter.split("_")[0].lower()
        out[f"{tag}_size_kib_per_launch"] = avg_kib
        out[f"copy_{tag}_size_kib"] = copy_kib
        out[f"{tag}_scale"] = scale
        out["launches_measured"] = len(kern)
        hbm += avg_kib * 1024.0 * scale
    out["hbm_bytes_per_launch"] = hbm
    launches = max(run["kernel_launches"], 1)
    out["kernel_ms_per_launch"] = run["kernel_ms"] / launches
    out["algorithmic_bytes_per_launch"] = run["kernel_algorithmic_bytes_per_launch"]
    out["hbm_gbs"] = hbm / (out["kernel_ms_per_launch"] * 1e-3) / 1e9
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", "sweep_kernel.h")
    with open(src, "rb") as fh:
        out["sweep_source_sha256"] = hashlib.sha256(fh.read()).hexdigest()
    with open(args.out, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
