"""HBM-traffic figures from rocprofv3 counter runs, for the benchmark line.

    python -m paper_2608_16960_amd.profiling FETCH_DIR WRITE_DIR BYTES_JSON OUT_TXT

FETCH_DIR / WRITE_DIR hold the counter_collection CSV of a `rocprofv3 --pmc
FETCH_SIZE` and a `--pmc WRITE_SIZE` run of `bench.py --calib-copy`; each
counter is scaled by what it reads for the plain 1 GiB device copy that run
makes.  BYTES_JSON is the bench line of the same run (for the kernel names).
The summary records, per kernel, the scaled bytes per dispatch and the SHA-1
of the kernel's source file, so that a figure is dropped once the source
changes.
"""
import csv
import glob
import hashlib
import json
import os
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {"k_fwd_sell<1>": "csrc/tsp_apply.hip", "k_adj_csc<1>": "csrc/tsp_apply.hip"}
COPY_KIB = 1 << 20  # the calibration copy moves 1 GiB each way


def source_sha(kernel):
    path = os.path.join(PKG, KERNEL_SOURCES[kernel])
    with open(path, "rb") as f:
        return hashlib.sha1(f.read()).hexdigest()[:12]


def _counter(dirname):
    path = glob.glob(os.path.join(dirname, "*counter_collection.csv"))[0]
    per = {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        key = None
        for k in KERNEL_SOURCES:
            if k.split("<")[0] in name:
                key = k
        if "copyBuffer" in name and float(r["Counter_Value"]) > 1e5:
            key = "copy"
        if key:
            per.setdefault(key, []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in per.items()}


def summarise(fetch_dir, write_dir):
    fe, wr = _counter(fetch_dir), _counter(write_dir)
    fs, ws = COPY_KIB / fe["copy"], COPY_KIB / wr["copy"]
    out = {}
    for k in KERNEL_SOURCES:
        if k in fe and k in wr:
            out[k] = {"fetch_kib": fe[k], "write_kib": wr[k], "fetch_scale": fs,
                      "write_scale": ws, "bytes": 1024.0 * (fe[k] * fs + wr[k] * ws),
                      "sha1": source_sha(k)}
    return out


def read_traffic(txt_path, kernel):
    """Scaled HBM bytes per dispatch of `kernel` from a summary file, or None
    when absent or taken on a different source of the kernel."""
    if not os.path.exists(txt_path):
        return None
    for line in open(txt_path):
        parts = line.split()
        if len(parts) == 4 and parts[0] == "traffic" and parts[1] == kernel:
            return float(parts[2]) if parts[3] == source_sha(kernel) else None
    return None


def main(argv):
    fetch_dir, write_dir, bench_json, out_txt = argv
    s = summarise(fetch_dir, write_dir)
    algo = {}
    if os.path.exists(bench_json):
        b = json.loads(open(bench_json).read().strip().splitlines()[-1])
        algo = {v["kernel"]: v["bytes"] for v in b["kernels"].values()}
    with open(out_txt, "a") as f:
        f.write("\n# machine-readable: traffic <kernel> <bytes per dispatch> <source sha1>\n")
        for k, v in s.items():
            f.write(f"traffic {k} {v['bytes']:.0f} {v['sha1']}\n")
            if k in algo:
                f.write(f"# {k}: fetch {v['fetch_kib']:.0f} KiB x {v['fetch_scale']:.3f}, write "
                        f"{v['write_kib']:.0f} KiB x {v['write_scale']:.3f}; algorithmic "
                        f"{algo[k]:.0f} bytes; ratio {v['bytes'] / algo[k]:.3f}\n")


if __name__ == "__main__":
    main(sys.argv[1:])
