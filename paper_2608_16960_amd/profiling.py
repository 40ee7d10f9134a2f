"""HBM-traffic and FP64 figures from rocprofv3 counter runs, for the benchmark line.

    python -m paper_2608_16960_amd.profiling FETCH_DIR WRITE_DIR BYTES_JSON OUT_TXT
    python -m paper_2608_16960_amd.profiling valu PMC_DIR STATS_DIR OUT_TXT
    python -m paper_2608_16960_amd.profiling occupancy PMC_DIR OUT_TXT KERNEL...
    python -m paper_2608_16960_amd.profiling stats STATS_DIR OUT_MD TITLE COMMAND [NOTE...]

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
import re
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = {"k_fwd_sell<1>": "csrc/tsp_apply.hip", "k_adj_csc<1>": "csrc/tsp_apply.hip",
                  "k_tile_y<1>": "csrc/tsp_apply.hip",
                  "k_otf_forward<4>": "csrc/tsp_trace.hip",
                  "k_otf_adjoint<4, false>": "csrc/tsp_trace.hip",
                  "k_otf_adjoint<4, true>": "csrc/tsp_trace.hip"}
FP64_PEAK_TFLOPS = 78.6  # MI355X vector FP64, published
COPY_KIB = 1 << 20  # the calibration copy moves 1 GiB each way


def source_sha(kernel):
    """SHA-1 of the kernel's source file and the shared internal header (and,
    for the tracing kernels, of the tracer header)."""
    h = hashlib.sha1()
    paths = [KERNEL_SOURCES[kernel], "csrc/tsp_internal.h"]
    if "otf" in kernel:
        paths.append("csrc/tsp_trace_core.h")
    for p in paths:
        with open(os.path.join(PKG, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def _tok(kernel):
    """A kernel name as one token of a machine-readable line ("k_x<4, true>" -> "k_x<4,true>")."""
    return kernel.replace(" ", "")


def _match(name, kernel):
    """rocprofv3 kernel name -> does it denote `kernel` ("k_x<4>")?"""
    base, _, targ = kernel.partition("<")
    return re.search(r"\b" + base + r"<" + targ.rstrip(">") + r"\b", name) is not None


def _per_dispatch(dirname, kernel):
    """Mean per dispatch of every counter of `kernel` in a counter_collection CSV."""
    path = glob.glob(os.path.join(dirname, "*counter_collection.csv"))[0]
    acc = {}
    for r in csv.DictReader(open(path)):
        if _match(r["Kernel_Name"], kernel):
            acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    return {k: sum(v) / len(v) for k, v in acc.items()}


def _mean_ns(stats_dir, kernel):
    path = glob.glob(os.path.join(stats_dir, "*kernel_stats.csv"))[0]
    for r in csv.DictReader(open(path)):
        if _match(r["Name"], kernel):
            return float(r["AverageNs"])
    return None


def summarise_valu(pmc_dir, stats_dir, kernels=("k_otf_forward<4>", "k_otf_adjoint<4, false>",
                                                 "k_otf_adjoint<4, true>")):
    """FP64 work per dispatch from SQ_INSTS_VALU_{ADD,MUL,FMA,TRANS}_F64 (wave
    instructions; x64 lanes, FMA counts 2 flops) and the kernel's mean duration
    from a --kernel-trace --stats run of the same command."""
    out = {}
    for k in kernels:
        c = _per_dispatch(pmc_dir, k)
        ns = _mean_ns(stats_dir, k)
        if not c or ns is None:
            continue
        flops = 64.0 * (c.get("SQ_INSTS_VALU_ADD_F64", 0) + c.get("SQ_INSTS_VALU_MUL_F64", 0)
                        + 2.0 * c.get("SQ_INSTS_VALU_FMA_F64", 0)
                        + c.get("SQ_INSTS_VALU_TRANS_F64", 0))
        out[k] = {"fp64_flops": flops, "ns": ns, "counters": c, "sha1": source_sha(k),
                  "tflops": flops / ns / 1e3, "frac": flops / ns / 1e3 / FP64_PEAK_TFLOPS}
    return out


def read_valu(txt_path, kernel):
    """(FP64 flops per dispatch, fraction of the FP64 peak) of `kernel` from a
    summary file, or None when absent or taken on a different source."""
    if not os.path.exists(txt_path):
        return None
    for line in open(txt_path):
        parts = line.split()
        if len(parts) == 5 and parts[0] == "valu" and parts[1] == _tok(kernel):
            return (float(parts[2]), float(parts[3])) if parts[4] == source_sha(kernel) else None
    return None


def _counter(dirname):
    path = glob.glob(os.path.join(dirname, "*counter_collection.csv"))[0]
    per = {}
    for r in csv.DictReader(open(path)):
        name = r["Kernel_Name"]
        key = None
        for k in KERNEL_SOURCES:
            if _match(name, k):
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
        if len(parts) == 4 and parts[0] == "traffic" and parts[1] == _tok(kernel):
            return float(parts[2]) if parts[3] == source_sha(kernel) else None
    return None


def main_valu(argv):
    pmc_dir, stats_dir, out_txt = argv
    s = summarise_valu(pmc_dir, stats_dir)
    with open(out_txt, "a") as f:
        f.write("\n# machine-readable: valu <kernel> <FP64 flops per dispatch> <fraction of "
                f"{FP64_PEAK_TFLOPS} TFLOP/s> <source sha1>\n")
        for k, v in s.items():
            f.write(f"valu {_tok(k)} {v['fp64_flops']:.0f} {v['frac']:.4f} {v['sha1']}\n")
            cs = ", ".join(f"{n} {x:.4g}" for n, x in sorted(v["counters"].items()))
            f.write(f"# {k}: {v['ns'] / 1e6:.2f} ms, {v['tflops']:.2f} TFLOP/s FP64; {cs}\n")


def _kernel_resources(pmc_dir, kernel):
    """(VGPRs, AGPRs, LDS bytes, workgroup size) of `kernel` from a counter_collection CSV."""
    path = glob.glob(os.path.join(pmc_dir, "*counter_collection.csv"))[0]
    for r in csv.DictReader(open(path)):
        if _match(r["Kernel_Name"], kernel):
            return (int(r["VGPR_Count"]), int(r.get("Accum_VGPR_Count") or 0),
                    int(r["LDS_Block_Size"]), int(r["Workgroup_Size"]))
    return None


def theoretical_waves_per_cu(vgpr, agpr, lds, wg):
    """Resident wavefronts per CU that registers and static LDS allow.  The
    counter CSV gives VGPRs in units of two (half of the allocation in the
    code object), so a SIMD holds 256 // (VGPRs + AGPRs) of them, at most 8;
    a CU has 4 SIMDs and 160 KiB of LDS (dynamic LDS is not in the CSV)."""
    regs = max(1, vgpr + agpr)
    per_simd = min(8, 256 // regs)
    waves_wg = max(1, wg // 64)
    by_regs = 4 * per_simd
    if lds <= 0:
        return by_regs
    by_lds = (160 * 1024 // lds) * waves_wg
    return min(by_regs, by_lds)


def main_occupancy(argv):
    pmc_dir, out_txt, *kernels = argv
    with open(out_txt, "a") as f:
        f.write("\n| kernel | VGPRs (CSV units) | AGPRs | static LDS bytes / workgroup | workgroup | "
                "resident waves per CU allowed (registers, static LDS) | MeanOccupancyPerCU (waves) "
                "| OccupancyPercent (of 32 waves) |\n|---|---|---|---|---|---|---|---|\n")
        for k in kernels:
            c = _per_dispatch(pmc_dir, k)
            res = _kernel_resources(pmc_dir, k)
            if not c or res is None:
                continue
            th = theoretical_waves_per_cu(*res)
            f.write(f"| `{k}` | {res[0]} | {res[1]} | {res[2]} | {res[3]} | {th} | "
                    f"{c.get('MeanOccupancyPerCU', float('nan')):.1f} | "
                    f"{c.get('OccupancyPercent', float('nan')):.1f}% |\n")
        f.write("\n# machine-readable: occupancy <kernel> <mean waves per CU> <source sha1>\n")
        for k in kernels:
            c = _per_dispatch(pmc_dir, k)
            if c and k in KERNEL_SOURCES:
                f.write(f"occupancy {_tok(k)} {c.get('MeanOccupancyPerCU', float('nan')):.2f} "
                        f"{source_sha(k)}\n")


def read_occupancy(path, kernel):
    """Mean resident wavefronts per CU of `kernel` from an occupancy summary
    (its machine-readable lines), or None when absent or taken on a different
    source of the kernel."""
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if len(parts) == 4 and parts[0] == "occupancy" and parts[1] == _tok(kernel):
            return float(parts[2]) if parts[3] == source_sha(kernel) else None
    return None


def main_stats(argv):
    """stats STATS_DIR OUT_MD TITLE COMMAND [NOTE...]: the kernel_stats.csv of a
    --kernel-trace --stats run as a markdown table (kernels by total time),
    with the command that made it and free-form notes."""
    stats_dir, out_md, title, command, *notes = argv
    path = glob.glob(os.path.join(stats_dir, "*kernel_stats.csv"))[0]
    rows = list(csv.DictReader(open(path)))
    with open(out_md, "w") as f:
        f.write(f"# {title}\n\nCommand (from the repository root, on one MI355X):\n\n```\n"
                f"{command}\n```\n\n")
        for n in notes:
            f.write(n + "\n")
        f.write("\n| kernel | calls | average (us) | min (us) | max (us) | share of GPU time |\n"
                "|---|---|---|---|---|---|\n")
        torch_calls, torch_share = 0, 0.0
        for r in rows:
            name = r["Name"].replace("(anonymous namespace)::", "")
            if re.match(r"^(void )?at::", name):  # PyTorch's own kernels: one line for all
                torch_calls += int(r["Calls"])
                torch_share += float(r["Percentage"])
                continue
            name = re.sub(r"^(void )?(tsp::)?", "", re.sub(r"\(.*$", "", name))
            f.write(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                    f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                    f"{float(r['Percentage']):.2f}% |\n")
        if torch_calls:
            f.write(f"| PyTorch's own kernels (all kinds) | {torch_calls} | | | | "
                    f"{torch_share:.2f}% |\n")


def main(argv):
    if argv and argv[0] == "stats":
        return main_stats(argv[1:])
    if argv and argv[0] == "valu":
        return main_valu(argv[1:])
    if argv and argv[0] == "occupancy":
        return main_occupancy(argv[1:])
    fetch_dir, write_dir, bench_json, out_txt = argv
    s = summarise(fetch_dir, write_dir)
    algo = {}
    if os.path.exists(bench_json):
        for line in reversed(open(bench_json).read().strip().splitlines()):
            if line.startswith("{") and '"kernels"' in line:
                b = json.loads(line)
                algo = {v["kernel"]: v["bytes"] for v in b["kernels"].values()}
                break
    with open(out_txt, "a") as f:
        f.write("\n# machine-readable: traffic <kernel> <bytes per dispatch> <source sha1>\n")
        for k, v in s.items():
            f.write(f"traffic {_tok(k)} {v['bytes']:.0f} {v['sha1']}\n")
            if k in algo:
                f.write(f"# {k}: fetch {v['fetch_kib']:.0f} KiB x {v['fetch_scale']:.3f}, write "
                        f"{v['write_kib']:.0f} KiB x {v['write_scale']:.3f}; algorithmic "
                        f"{algo[k]:.0f} bytes; ratio {v['bytes'] / algo[k]:.3f}\n")


if __name__ == "__main__":
    main(sys.argv[1:])
