"""Benchmark of the spherical-grid projector on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload medium]
                    [--no-cpu-baseline]

A step is one forward projection y = F rho (stored segment lists) followed by
one deterministic adjoint x = F^T y, on the Medium workload: 50x50x50 grid,
30 cone-beam views of 256x256 pixels (1,966,080 rays), float32 object with an
exponential background and five Gaussian blobs (synthetic; the paper's own
data is not available).  Steps 1-3 of the method (the trace that builds the
segment stores) run once before timing, as in the paper's precompute; their
time is reported separately.

Prints ONE JSON line: rays/s of forward+adjoint as `value`, segments/s and
per-kernel roofline fractions alongside, the CPU FP64 oracle timed on the host
cores on a bounded sample, and the trace time.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def _args():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--workload", default="medium", choices=["medium", "tiny", "learned", "diff"])
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--calib-copy", action="store_true",
                   help="after timing, run a plain 1 GiB device copy (counter calibration)")
    p.add_argument("--cpu-views", type=int, default=30,
                   help="views of the workload the CPU oracle traces (bounded sample)")
    return p.parse_args()


def cpu_baseline(w, n_views):
    """The FP64 oracle as it stands, on the host cores, on a subset of views:
    trace (steps 1-3) and apply (forward + adjoint from its own lists) timed
    separately; `value` is the apply rate in rays/s, like the GPU's."""
    import numpy as np

    import oracle
    v = w.views
    sel = np.linspace(0, v.n_views - 1, n_views).round().astype(int)
    s, d = oracle.cone_rays(v.pos[sel], v.look[sel], v.up[sel], v.fov_deg[sel], v.H, v.W)
    t0 = time.perf_counter()
    tr = oracle.trace(w.grid.arrays(), s, d)
    t1 = time.perf_counter()
    rho = w.rho[0].astype(np.float64)
    y = oracle.forward(tr, rho)
    t2 = time.perf_counter()
    oracle.adjoint(tr, y, w.grid.size)
    t3 = time.perf_counter()
    R = len(s)
    S = int(tr["counts"].sum())
    return {
        "value": R / (t3 - t1), "unit": "rays/s", "cores": oracle.num_threads(), "kind": "oracle",
        "sample": f"{len(sel)} of {v.n_views} views ({R} rays, {S} segments) of the "
                  f"{w.name} workload; forward (OpenMP) + adjoint (serial) from the oracle's "
                  f"own segment lists, FP64",
        "segments_per_s": S / (t3 - t1),
        "trace_rays_per_s": R / (t1 - t0),
        "trace_s": t1 - t0, "forward_s": t2 - t1, "adjoint_s": t3 - t2,
        "host": platform.processor() or platform.machine(),
    }


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py: this build measures one GPU only (asked for --gpus {a.gpus}); "
              "the projector shards by views across GPUs by design but no multi-GPU path "
              "is built.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    w = getattr(W, a.workload)()
    rho = torch.from_numpy(w.rho[:1]).to(dev)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Projector(w.grid, views=w.views, mode="csr")
    torch.cuda.synchronize()
    trace_s = time.perf_counter() - t0
    info = P.info()
    R, V, S, B = info["n_rays"], info["n_voxels"], info["n_segments"], 1

    y = torch.empty((1, *P.out_shape), dtype=torch.float32, device=dev)
    x = torch.empty((1, *P.shape), dtype=torch.float32, device=dev)

    def step():
        P.forward(rho, out=y)
        P.backproject(y, "deterministic", out=x)

    for _ in range(a.warmup):
        step()
    K = a.steps
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(K)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(K):
        e0, e1, e2 = ev[k]
        e0.record()
        P.forward(rho, out=y)
        e1.record()
        P.backproject(y, "deterministic", out=x)
        e2.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    fwd_ms = sum(e[0].elapsed_time(e[1]) for e in ev) / K
    adj_ms = sum(e[1].elapsed_time(e[2]) for e in ev) / K
    ms_step = wall / K * 1e3

    # algorithmic bytes per launch (4-byte index + 4-byte length per segment,
    # 8 bytes of row / column bookkeeping, object and measurements once)
    fwd_bytes = 8 * S + 8 * R + 4 * B * R + 4 * B * V
    adj_bytes = 8 * S + 8 * V + 4 * B * V + 4 * B * R
    kern = {
        "forward": {"kernel": "k_fwd_sell<1>", "ms": fwd_ms, "bytes": fwd_bytes,
                    "GBps": fwd_bytes / fwd_ms / 1e6},
        "adjoint": {"kernel": "k_adj_csc<1>", "ms": adj_ms, "bytes": adj_bytes,
                    "GBps": adj_bytes / adj_ms / 1e6},
    }
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    line = {
        "metric": "rays/s & segments/s fwd+adjoint (%HBM roofline); projector calls to residual",
        "value": R / (ms_step / 1e3),
        "unit": "rays/s",
        "n_gpus": 1, "steps": K, "warmup": a.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (f64 geometry)", "data": "synthetic",
        "config": {"workload": f"{w.name}: grid {P.shape}, {w.views.n_views} cone views "
                               f"{w.views.H}x{w.views.W}, {R} rays, {S} segments, batch 1",
                   "mode": "csr + voxel-major deterministic adjoint"},
        "segments_per_s": S / (ms_step / 1e3),
        "roofline": {"bound": "hbm", "achieved": d["GBps"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": d["GBps"] / HBM_PEAK_GBS, "traffic": None, "kernel": d["kernel"]},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in kern.items()},
        "trace_s": trace_s,
        "stored_slots": info["n_stored"], "pad_frac": info["n_stored"] / max(S, 1) - 1,
    }
    if a.calib_copy:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        line["calib_copy_bytes_each_way"] = src.numel() * 4
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, a.cpu_views)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
