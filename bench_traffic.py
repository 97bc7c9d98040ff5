"""HBM traffic per kernel launch from rocprofv3 counter runs, for bench.py's roofline.

Two counter runs of the same bench command (FETCH_SIZE, then WRITE_SIZE; each in KiB per
dispatch) and the same two counters for a plain device copy of known size (bench.py
--copy-probe MiB) give the scale factors: true bytes = factor * counter * 1024, with the
factor set so that the copy reads and writes exactly its size. Writes, per workload and
bench stage, the mean bytes per launch of the kernel the stage ran, the kernel's name and
a hash of its source file (bench.py ignores a record whose source has changed since).

    python bench_traffic.py --workload pm256 --fetch F.csv --write W.csv \
        --copy-fetch CF.csv --copy-write CW.csv --copy-mib 256 --command "..." \
        --out profiles/traffic.json
"""
import argparse
import csv
import json
import os
import re

from bench import KERNEL_SOURCES, source_sha

# kernel function name (without template arguments) -> bench stage
STAGE_OF = {
    "fill_zero_kernel": "zero_mesh", "deposit_kernel": "cic_deposit",
    "deposit_tiled_kernel": "cic_deposit", "fwd_z_kernel": "fft_fwd_z",
    "fwd_y_kernel": "fft_fwd_y", "fwd_x_bin_kernel": "fft_fwd_x_bin",
    "response_kernel": "nu_response",
    "inv_x_kernel": "inv_x_green", "inv_y_kernel": "fft_inv_y", "inv_z_kernel": "fft_inv_z",
    "interp_kernel": "cic_interp", "interp_tiled_kernel": "cic_interp",
    "deposit_patch_kernel": "cic_deposit", "patch_reduce_kernel": "patch_reduce",
    "kick_drift_kernel": "kick_drift", "patch_fwd_z_kernel": "patch_fwd_z",
    "inv_xy_kernel": "inv_xy_green", "fwd_zy_kernel": "fft_fwd_zy",
    "inv_yz_kernel": "inv_yz",
}


def kernel_short(name):
    m = re.search(r"pmnu::\(anonymous namespace\)::(\w+)(<[^(]*>)?\(", name)
    return (m.group(1), m.group(1) + (m.group(2) or "")) if m else (None, None)


def per_kernel(path, counter):
    """{kernel with template args: [values per dispatch]} for one counter."""
    out = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] != counter:
                continue
            base, full = kernel_short(r["Kernel_Name"])
            if base in STAGE_OF:
                out.setdefault(full, []).append(float(r["Counter_Value"]))
    return out


def largest_copy(path, counter):
    best = None
    with open(path) as f:
        for r in csv.DictReader(f):
            if r["Counter_Name"] == counter and "copyBuffer" in r["Kernel_Name"]:
                v = float(r["Counter_Value"])
                best = v if best is None else max(best, v)
    if best is None:
        raise SystemExit(f"no copy dispatch with {counter} in {path}")
    return best


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--fetch", required=True)
    ap.add_argument("--write", required=True)
    ap.add_argument("--copy-fetch", required=True)
    ap.add_argument("--copy-write", required=True)
    ap.add_argument("--copy-mib", type=float, required=True)
    ap.add_argument("--command", default="")
    ap.add_argument("--out", required=True)
    a = ap.parse_args()
    size = a.copy_mib * (1 << 20)
    f_fac = size / (largest_copy(a.copy_fetch, "FETCH_SIZE") * 1024)
    w_fac = size / (largest_copy(a.copy_write, "WRITE_SIZE") * 1024)
    fetch, write = per_kernel(a.fetch, "FETCH_SIZE"), per_kernel(a.write, "WRITE_SIZE")
    table = {}
    if os.path.exists(a.out):
        with open(a.out) as f:
            table = json.load(f)
    rec = {}
    for full in sorted(set(fetch) & set(write)):
        stage = STAGE_OF[full.split("<")[0]]
        fb = f_fac * 1024 * sum(fetch[full]) / len(fetch[full])
        wb = w_fac * 1024 * sum(write[full]) / len(write[full])
        rec.setdefault(stage, {})[full] = {
            "bytes_per_launch": fb + wb, "fetch_bytes": fb, "write_bytes": wb,
            "dispatches": len(fetch[full]), "source_sha": source_sha(KERNEL_SOURCES[stage])}
    table[a.workload] = {"calibration": {"copy_mib": a.copy_mib, "fetch_factor": f_fac,
                                         "write_factor": w_fac},
                         "command": a.command, "kernels": rec}
    with open(a.out, "w") as f:
        json.dump(table, f, indent=1, sort_keys=True)
    print(json.dumps({"fetch_factor": f_fac, "write_factor": w_fac,
                      "stages": {s: {k: round(v["bytes_per_launch"] / 1e6, 2)
                                     for k, v in d.items()} for s, d in rec.items()}}))


if __name__ == "__main__":
    main()
