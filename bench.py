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
cores, and the trace time.  Unless --quick, it also measures (as extra fields)
the on-the-fly mode on the Large workload (batch 4, no segment storage), the
stored-list path on the Differentiation workload, the attenuated emission
model on Medium, and the learned warm start (projector calls to reach the
plain solver's residual, 200 held-out phantoms).
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
    p.add_argument("--quick", action="store_true",
                   help="only the Medium forward+adjoint line (for profiler runs)")
    p.add_argument("--calib-copy", action="store_true",
                   help="after timing, run a plain 1 GiB device copy (counter calibration)")
    p.add_argument("--large-only", action="store_true",
                   help="only the Large on-the-fly forward and adjoint (for counter runs)")
    p.add_argument("--extras", default="all",
                   help="comma-separated extra workloads after the Medium line (tiny, "
                        "cnn_layers, onthefly_large, stored_large, diff_csr, "
                        "explicit_rays_medium, attenuated_medium, learned_warm_start) or 'all'")
    p.add_argument("--cpu-views", type=int, default=30,
                   help="views of the workload the CPU oracle traces (bounded sample)")
    p.add_argument("--cpu-full", action="store_true",
                   help="CPU oracle on all 100 Differentiation views (minutes, ~46 GB of "
                        "host memory) instead of 10")
    return p.parse_args()


def _host():
    """CPU model (lscpu, else /proc/cpuinfo) with lscpu's vendor, family,
    model, stepping, clock and cache lines where it prints them (a virtual
    machine may name the CPU only by its brand), logical CPUs, and the CPUs
    this process may run on."""
    import subprocess
    model = None
    lscpu = {}
    keys = ("Vendor ID", "CPU family", "Model", "Stepping", "CPU max MHz", "BogoMIPS",
            "L2 cache", "L3 cache", "Hypervisor vendor")
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() == "Model name":
                model = v.strip()
            elif k.strip() in keys:
                lscpu[k.strip()] = v.strip()
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for line in open("/proc/cpuinfo"):
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        except OSError:
            model = platform.processor() or platform.machine()
    return {"model": model, "lscpu": lscpu, "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0))}


def cpu_baseline(w, n_views, large_views=6, diff_views=10, full=False):
    """The FP64 oracle as it stands, on the host cores: trace (steps 1-3) and
    apply (forward + adjoint from its own lists) timed separately, mirroring
    the paper's precompute / raytrace split.  The forward runs on all OpenMP
    threads; the oracle's adjoint is a plain serial loop and is timed as such.
    `value` is the apply rate in rays/s over `n_views` views of the workload,
    like the GPU's.  Also: one thread; the Learned geometry in full (trace
    once, apply on the whole configuration); the Differentiation workload on
    `diff_views` of its 100 views (all of them with full=True: about 2.3e9
    segments, 46 GB of host memory); and a fixed subset of the Large workload
    (every 30th view)."""
    import numpy as np

    import oracle
    from paper_2608_16960_amd import workloads as W

    def run(grid, v, sel, rho):
        s, d = oracle.cone_rays(v.pos[sel], v.look[sel], v.up[sel], v.fov_deg[sel], v.H, v.W)
        t0 = time.perf_counter()
        tr = oracle.trace(grid.arrays(), s, d)
        t1 = time.perf_counter()
        y = oracle.forward(tr, rho)
        t2 = time.perf_counter()
        oracle.adjoint(tr, y, grid.size)
        t3 = time.perf_counter()
        return tr, len(s), int(tr["counts"].sum()), (t1 - t0, t2 - t1, t3 - t2)

    def leg(name, grid, v, sel, rho):
        _log(f"cpu baseline: {name}")
        tr, R, S, (ts, fs, as_) = run(grid, v, sel, rho)
        del tr
        return {"views": f"{len(sel)} of {v.n_views}", "rays": R, "segments": S,
                "trace_s": ts, "forward_s": fs, "adjoint_s": as_,
                "trace_rays_per_s": R / ts, "apply_rays_per_s": R / (fs + as_),
                "apply_segments_per_s": S / (fs + as_)}

    nt = oracle.num_threads()
    v = w.views
    sel = np.linspace(0, v.n_views - 1, n_views).round().astype(int)
    rho = w.rho[0].reshape(-1).astype(np.float64)
    _log("cpu baseline: main workload")
    tr, R, S, (ts, fs, as_) = run(w.grid, v, sel, rho)
    out = {
        "value": R / (fs + as_), "unit": "rays/s", "cores": nt, "kind": "oracle",
        "sample": f"{len(sel)} of {v.n_views} views ({R} rays, {S} segments) of the "
                  f"{w.name} workload; forward on {nt} OpenMP threads + adjoint on one thread "
                  f"(the oracle's adjoint loop is serial), from the oracle's own segment "
                  f"lists, FP64",
        "segments_per_s": S / (fs + as_),
        "trace_rays_per_s": R / ts,
        "trace_s": ts, "forward_s": fs, "adjoint_s": as_, "adjoint_threads": 1,
        "host": _host(),
    }
    # one thread: apply on the same lists; trace on the first view only
    oracle.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.forward(tr, rho)
        f1 = time.perf_counter() - t0
        del tr
        _, R1, _, (t1s, _, _) = run(w.grid, v, sel[:1], rho)
    finally:
        oracle.set_num_threads(nt)
    out["one_thread"] = {"apply_rays_per_s": R / (f1 + as_), "forward_s": f1,
                         "trace_rays_per_s": R1 / t1s, "trace_sample": f"1 view ({R1} rays)"}
    # Learned geometry, whole configuration (first training phantom)
    g, lv = W.learned_geometry()
    lrho = W.learned_phantoms(g, 1, seed=6)[0].reshape(-1).astype(np.float64)
    out["learned_full"] = leg("learned", g, lv, np.arange(lv.n_views), lrho)
    # Differentiation workload (views spread over the orbit)
    D = W.diff()
    nd = D.views.n_views if full else diff_views
    dsel = np.linspace(0, D.views.n_views - 1, nd).round().astype(int)
    out["diff_full" if full else "diff_subset"] = leg(
        "differentiation", D.grid, D.views, dsel, D.rho[0].reshape(-1).astype(np.float64))
    del D
    # Large subset, all threads
    L = W.large()
    lsel = np.arange(0, L.views.n_views, L.views.n_views // large_views)[:large_views]
    out["large_subset"] = dict(leg("large", L.grid, L.views, lsel,
                                   L.rho[0].reshape(-1).astype(np.float64)),
                               view_ids=lsel.tolist(), object="first of 4")
    return out


def measured_stream_gbps(dev, nbytes=1 << 30, reps=10):
    """HBM rates of plain streams of `nbytes` on this device: the library's
    hand-written non-temporal copy (bytes read + written per second) and
    read, each at its best grid size of a few, and torch's copy for
    reference."""
    import torch

    from paper_2608_16960_amd import nn as NN
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    part = torch.empty(1 << 16, dtype=torch.float32, device=dev)
    out = {}
    for blocks in (1024, 2048, 4096, 8192, 16384):
        c = _time_ms(lambda: NN.stream_copy(src, dst, blocks), reps)
        r = _time_ms(lambda: NN.stream_read(src, part, blocks), reps)
        out.setdefault("copy", []).append((2.0 * nbytes / c / 1e6, blocks))
        out.setdefault("read", []).append((nbytes / r / 1e6, blocks))
    assert torch.equal(dst[:1024], src[:1024])
    t = _time_ms(lambda: dst.copy_(src), reps)
    del src, dst, part
    best_c, best_r = max(out["copy"]), max(out["read"])
    return {"copy_GBps": best_c[0], "copy_blocks": best_c[1],
            "read_GBps": best_r[0], "read_blocks": best_r[1],
            "torch_copy_GBps": 2.0 * nbytes / t / 1e6, "bytes": nbytes}


def _log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _kernel_ms(P, fn, reps, warm=1):
    """Mean duration of the main kernel of P's call fn (a forward or an
    adjoint), from the HIP events the library records around it on the
    call's stream (tsp_set_timing_events); the calls run back to back."""
    import torch
    for _ in range(warm):
        fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, b in evs:
        a.record()
        b.record()
    torch.cuda.synchronize()
    for a, b in evs:
        P.set_timing_events(a, b)
        fn()
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / reps


def _time_ms(fn, reps, warm=1):
    import torch
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def extra_tiny(reps=200):
    """Tiny workload (latency-bound: about 1e5 segments): time per launch of
    the stored-list forward and deterministic adjoint."""
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector
    w = W.tiny()
    P = Projector(w.grid, views=w.views)
    rho = torch.from_numpy(w.rho).cuda()
    y = P.forward(rho)
    x = torch.empty_like(rho)
    f_ms = _time_ms(lambda: P.forward(rho, out=y), reps, warm=5)
    a_ms = _time_ms(lambda: P.backproject(y, "deterministic", out=x), reps, warm=5)
    inf = P.info()
    P.close()
    return {"workload": f"tiny: grid {P.shape}, {w.views.n_views} cone views "
                        f"{w.views.H}x{w.views.W}, {inf['n_rays']} rays, {inf['n_segments']} "
                        f"segments, batch 1",
            "forward_us": f_ms * 1e3, "adjoint_us": a_ms * 1e3, "step_us": (f_ms + a_ms) * 1e3,
            "note": "latency-bound (under 1 MB moved); time only"}


def extra_cnn(reps=20):
    """The 32 -> 32 convolution kernels (BF16 MFMA, FP32 accumulation) at the
    training shape, batch 8 of 64 x 32 x 64 voxels: forward, input gradient
    and weight gradient (with the bias gradient), each 2 * 27 * 32 * 32
    flop per voxel, against the dense BF16 peak."""
    import torch

    from paper_2608_16960_amd import nn as NN
    N, D = 8, (64, 32, 64)
    g = torch.Generator(device="cpu").manual_seed(3)
    x = torch.randn((N, *D, 32), generator=g).to(torch.bfloat16).cuda()
    dz = torch.randn((N, *D, 32), generator=g).to(torch.bfloat16).cuda()
    w = (0.05 * torch.randn((27, 32, 32), generator=g)).to(torch.bfloat16).cuda()
    b = torch.zeros(32, device="cuda")
    out = torch.empty_like(x)
    dw = torch.empty((27, 32, 32), device="cuda")
    db = torch.empty(32, device="cuda")
    ws = torch.empty(int(NN.lib.tspnn_conv_workspace(N, *D)) // 4 + 1, device="cuda")
    p, s = NN._p, NN._s
    fwd = lambda: NN.check(NN.lib.tspnn_conv_fwd(p(x), N, *D, p(w), p(b), p(out), s()))
    bwd_d = lambda: NN.check(NN.lib.tspnn_conv_bwd_data(p(dz), N, *D, p(w), p(x), p(out), s()))
    bwd_w = lambda: NN.check(NN.lib.tspnn_conv_bwd_weight(p(x), p(dz), N, *D, p(dw), p(db),
                                                          p(ws), s()))
    flops = 2.0 * 27 * 32 * 32 * N * D[0] * D[1] * D[2]
    res = {}
    for name, kern, fn in (("forward", "k_conv_lds<0>", fwd),
                           ("input_gradient", "k_conv_lds<1>", bwd_d),
                           ("weight_gradient", "k_conv_wgrad_tiled", bwd_w)):
        ms = _time_ms(fn, reps, warm=3)
        tf = flops / ms / 1e9
        res[name] = {"kernel": kern, "us": ms * 1e3, "TFLOPs": tf, "frac_of_bf16_peak": tf / 2500.0}
    return {"workload": "batch 8 of 64x32x64 voxels, 32 -> 32 channels, 3x3x3 taps",
            "flop_per_launch": flops, "peak_TFLOPs": 2500.0, **res}


def extra_large_onthefly():
    """Large workload on the fly, batch 4: count pass (steps 1-3 without
    storage), forward and atomic adjoint per launch; the fixed-point
    (reproducible) adjoint per launch; and the deterministic adjoint, traced
    chunk by chunk within each call (second call timed, the first one
    allocates its working memory)."""
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector
    w = W.large()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Projector(w.grid, views=w.views, mode="onthefly")
    torch.cuda.synchronize()
    count_s = time.perf_counter() - t0
    inf = P.info()
    R, V, S, B = inf["n_rays"], inf["n_voxels"], inf["n_segments"], 4
    rho = torch.from_numpy(w.rho).cuda()
    y = P.forward(rho)
    x = torch.empty_like(rho)
    f_ms = _time_ms(lambda: P.forward(rho, out=y), 3)
    a_ms = _time_ms(lambda: P.backproject(y, "atomic", out=x), 2)
    fx_ms = _time_ms(lambda: P.backproject(y, "fixedpoint", out=x), 2)
    P.backproject(y, "deterministic", out=x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.backproject(y, "deterministic", out=x)
    torch.cuda.synchronize()
    det_s = time.perf_counter() - t0
    alg = 4 * B * V + 4 * B * R
    P.close()
    from paper_2608_16960_amd.profiling import read_valu
    fp64 = {}
    for k, kern in (("forward", "k_otf_forward<4>"), ("adjoint", "k_otf_adjoint<4, false>"),
                    ("fixedpoint_adjoint", "k_otf_adjoint<4, true>")):
        r = read_valu(os.path.join(ROOT, "profiles", "otf_large_fp64.txt"), kern)
        fp64[k] = None if r is None else {
            "flops_per_launch": r[0], "frac_of_fp64_peak": r[1],
            "tflops_live": r[0] / ({"forward": f_ms, "adjoint": a_ms,
                                    "fixedpoint_adjoint": fx_ms}[k] * 1e9)}
    return {"workload": f"large: grid {P.shape}, {w.views.n_views} cone views "
                        f"{w.views.H}x{w.views.W}, {R} rays, {S} segments, batch {B}",
            "count_s": count_s, "forward_ms": f_ms, "adjoint_ms": a_ms,
            "deterministic_adjoint_s": det_s, "fixedpoint_adjoint_ms": fx_ms,
            "forward_rays_per_s": B * R / f_ms * 1e3, "forward_segments_per_s": B * S / f_ms * 1e3,
            "adjoint_rays_per_s": B * R / a_ms * 1e3, "adjoint_segments_per_s": B * S / a_ms * 1e3,
            "forward_hbm_frac": alg / f_ms / 1e6 / HBM_PEAK_GBS,
            "fp64_valu": fp64,
            "note": "FP64 tracing per launch; the HBM roof does not bind (4BV + 4BR bytes); "
                    "fp64_valu from rocprofv3 FP64 instruction counters (profiles)"}


def extra_large_csr(reps=5):
    """Large workload from stored segment lists: on one MI355X the ray-major
    and voxel-major stores (about 5 bytes per segment each, 8.46e9 segments)
    fit in HBM, the transpose sorted in passes that fit the rest; batch 4,
    deterministic adjoint."""
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector
    w = W.large()
    torch.cuda.empty_cache()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Projector(w.grid, views=w.views)
    torch.cuda.synchronize()
    trace_s = time.perf_counter() - t0
    inf = P.info()
    R, V, S, B = inf["n_rays"], inf["n_voxels"], inf["n_segments"], 4
    rho = torch.from_numpy(w.rho).cuda()
    y = P.forward(rho)
    x = torch.empty_like(rho)
    f_ms = _time_ms(lambda: P.forward(rho, out=y), reps)
    a_ms = _time_ms(lambda: P.backproject(y, "deterministic", out=x), reps)
    fk = _kernel_ms(P, lambda: P.forward(rho, out=y), reps)
    ak = _kernel_ms(P, lambda: P.backproject(y, "deterministic", out=x), reps)
    fb, ab = 8 * S + 8 * R + 4 * B * R + 4 * B * V, 8 * S + 8 * V + 4 * B * V + 4 * B * R
    P.close()
    del y, x, rho
    torch.cuda.empty_cache()
    return {"workload": f"large from stored lists: {R} rays, {S} segments, batch {B}",
            "trace_s": trace_s, "device_GB": inf["device_bytes"] / 1e9,
            "forward_ms": f_ms, "adjoint_ms": a_ms,
            # the main kernels alone (k_fwd_sell<4>, k_adj_csc<4>)
            "forward_kernel_ms": fk, "adjoint_kernel_ms": ak,
            "forward_kernel_hbm_frac": fb / fk / 1e6 / HBM_PEAK_GBS,
            "adjoint_kernel_hbm_frac": ab / ak / 1e6 / HBM_PEAK_GBS,
            "forward_rays_per_s": B * R / f_ms * 1e3, "adjoint_rays_per_s": B * R / a_ms * 1e3,
            "forward_hbm_frac": fb / f_ms / 1e6 / HBM_PEAK_GBS,
            "adjoint_hbm_frac": ab / a_ms / 1e6 / HBM_PEAK_GBS}


def extra_diff_csr():
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector
    w = W.diff()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Projector(w.grid, views=w.views)
    torch.cuda.synchronize()
    trace_s = time.perf_counter() - t0
    inf = P.info()
    R, V, S = inf["n_rays"], inf["n_voxels"], inf["n_segments"]
    rho = torch.from_numpy(w.rho).cuda()
    y = P.forward(rho)
    x = torch.empty_like(rho)
    # the main kernels alone (k_fwd_sell<1>, k_adj_csc<1>), as the step's
    # roofline takes them; the whole calls beside them
    f_ms = _kernel_ms(P, lambda: P.forward(rho, out=y), 10)
    a_ms = _kernel_ms(P, lambda: P.backproject(y, "deterministic", out=x), 10)
    f_call = _time_ms(lambda: P.forward(rho, out=y), 10)
    a_call = _time_ms(lambda: P.backproject(y, "deterministic", out=x), 10)
    fb, ab = 8 * S + 8 * R + 4 * R + 4 * V, 8 * S + 8 * V + 4 * V + 4 * R
    P.close()
    torch.cuda.empty_cache()
    from paper_2608_16960_amd.profiling import read_traffic
    tf = os.path.join(ROOT, "profiles", "hbm_traffic_diff.txt")
    traffic = {k: read_traffic(tf, kern) for k, kern in (("forward", "k_fwd_sell<1>"),
                                                           ("adjoint", "k_adj_csc<1>"))}
    return {"workload": f"diff: grid {P.shape}, {w.views.n_views} cone views "
                        f"{w.views.H}x{w.views.W}, {R} rays, {S} segments, batch 1",
            "trace_s": trace_s, "forward_ms": f_ms, "adjoint_ms": a_ms,
            "forward_call_ms": f_call, "adjoint_call_ms": a_call,
            "rays_per_s": R / (f_call + a_call) * 1e3,
            "segments_per_s": S / (f_call + a_call) * 1e3,
            "forward_hbm_frac": fb / f_ms / 1e6 / HBM_PEAK_GBS,
            "adjoint_hbm_frac": ab / a_ms / 1e6 / HBM_PEAK_GBS,
            "forward_traffic_frac": None if traffic["forward"] is None
            else traffic["forward"] / f_ms / 1e6 / HBM_PEAK_GBS,
            "adjoint_traffic_frac": None if traffic["adjoint"] is None
            else traffic["adjoint"] / a_ms / 1e6 / HBM_PEAK_GBS,
            "traffic_bytes": traffic}


def extra_atten_medium(reps=10):
    """Attenuated emission model (Sec. 9.3) on the Medium workload: one
    forward (sunward optical depths, then the line-of-sight pass with the
    running absorption) and one backward per call, batch 1."""
    import numpy as np
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.atten import Attenuated
    from paper_2608_16960_amd.projector import Projector
    w = W.medium()
    P = Projector(w.grid, views=w.views)
    sig = torch.from_numpy(np.random.default_rng(70).uniform(0.02, 0.3, w.grid.shape)
                           .astype(np.float32))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = Attenuated(P, sig, [0.0, 1.0, 0.0])
    torch.cuda.synchronize()
    sun_s = time.perf_counter() - t0
    rho = torch.from_numpy(w.rho).cuda()
    y, tau = M.forward(rho, keep_tau=True)
    gy = torch.randn_like(y)
    f_ms = _time_ms(lambda: M.forward(rho, keep_tau=True), reps)
    b_ms = _time_ms(lambda: M.backward(rho, tau, gy, "deterministic"), reps)
    ba_ms = _time_ms(lambda: M.backward(rho, tau, gy, "atomic"), reps)
    inf, infs = P.info(), M.sun.info()
    R = inf["n_rays"]
    out = {"workload": f"medium with attenuation: {R} lines of sight, {inf['n_voxels']} sunward "
                       f"rays, {inf['n_segments']} + {infs['n_segments']} segments, batch 1",
           "sun_trace_s": sun_s, "forward_ms": f_ms, "backward_ms": b_ms,
           "backward_atomic_ms": ba_ms,
           "forward_rays_per_s": R / f_ms * 1e3, "forward_backward_rays_per_s": R / (f_ms + b_ms) * 1e3}
    P.close()
    M.sun.close()
    return out


def extra_explicit_medium(reps=10):
    """Custom view geometry at scale (Sec. 4.2, Listing 4): the Medium
    workload's 1,966,080 rays handed over as explicit start / direction
    arrays instead of cone views; trace, forward and deterministic adjoint."""
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector
    w = W.medium()
    Pc = Projector(w.grid, views=w.views, csc=False)
    s, d = (t.cpu().numpy() for t in Pc.rays())
    Pc.close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P = Projector(w.grid, rays=(s, d))
    torch.cuda.synchronize()
    trace_s = time.perf_counter() - t0
    rho = torch.from_numpy(w.rho).cuda()
    y = P.forward(rho)
    x = torch.empty_like(rho)
    f_ms = _time_ms(lambda: P.forward(rho, out=y), reps)
    a_ms = _time_ms(lambda: P.backproject(y, "deterministic", out=x), reps)
    R = P.info()["n_rays"]
    P.close()
    return {"workload": f"medium as {R} explicit rays", "trace_s": trace_s, "forward_ms": f_ms,
            "adjoint_ms": a_ms, "rays_per_s": R / (f_ms + a_ms) * 1e3}


def extra_learned(epochs=12):
    import numpy as np
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.learned import WarmStart
    from paper_2608_16960_amd.projector import Projector
    g, v = W.learned_geometry()
    P = Projector(g, views=v)
    ws = WarmStart(P, k0=2, K=60)
    train = torch.from_numpy(W.learned_phantoms(g, 2000, seed=6)).cuda()
    xs = []
    for b0 in range(0, train.shape[0], 8):
        xs.append(ws.inputs(ws.measure(train[b0:b0 + 8]))[0])
    x_in = torch.cat(xs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = ws.fit(x_in, train, epochs=epochs, batch=8, lr=2e-3)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    del x_in, train
    res = ws.evaluate(torch.from_numpy(W.learned_phantoms(g, 200, seed=7)).cuda(), curves=True)
    warm = np.array(res["warm_calls"])
    plain = np.array(res["plain_calls"])
    P.close()
    return {"workload": "learned: grid (64, 32, 64), 64 cone views 256x256; 2000 training and "
                        "200 held-out phantoms",
            "plain_calls_median": float(np.median(plain)),
            "warm_calls_median": float(np.median(warm)),
            "warm_calls_p90": float(np.percentile(warm, 90)), "warm_calls_max": int(warm.max()),
            "fallback_rate": float(np.mean(res["fallback"])),
            "reduction": float(np.median(plain) / np.median(warm)),
            "train_epochs": epochs, "train_s": train_s, "train_mse_last": hist[-1],
            # median over the held-out phantoms of residual / R* against
            # projector calls: plain GD from zero, and the warm start (4 input
            # calls + 1 for the CNN output's residual, then GD)
            "curves": res["curves"]}


def main():
    a = _args()
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); "
              "the projector shards by views across GPUs by design but no multi-GPU path "
              "is built.", file=sys.stderr)
        sys.exit(2)
    if a.steps < 2 and not a.large_only:
        print("bench.py needs --steps 2 or more: alternate steps time the forward's and the "
              "adjoint's kernels", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2608_16960_amd import workloads as W
    from paper_2608_16960_amd.projector import Projector

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    if a.large_only:
        print(json.dumps({"onthefly_large": extra_large_onthefly()}))
        return
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
    # The library records a pair of HIP events just before and just after a
    # call's main kernel, on the call's stream (tsp_set_timing_events): even
    # steps time the forward's kernel, odd steps the adjoint's, so each step
    # carries two event records (each adds a few microseconds between
    # launches).  The events are created by a first record before the timed
    # region.
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(K)]
    for e in ev:
        for t in e:
            t.record()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(K):
        s0, s1 = ev[k]
        if k % 2 == 0:
            P.set_timing_events(s0, s1)
        P.forward(rho, out=y)
        if k % 2 == 1:
            P.set_timing_events(s0, s1)
        P.backproject(y, "deterministic", out=x)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    fwd_t = sorted(ev[k][0].elapsed_time(ev[k][1]) for k in range(0, K, 2))
    adj_t = sorted(ev[k][0].elapsed_time(ev[k][1]) for k in range(1, K, 2))
    fwd_ms, adj_ms = sum(fwd_t) / len(fwd_t), sum(adj_t) / len(adj_t)
    ms_step = wall / K * 1e3
    # algorithmic bytes per launch (4-byte index + 4-byte length per segment,
    # 8 bytes of row / column bookkeeping, object and measurements once)
    fwd_bytes = 8 * S + 8 * R + 4 * B * R + 4 * B * V
    adj_bytes = 8 * S + 8 * V + 4 * B * V + 4 * B * R
    # the kernels' own mean durations (the adjoint's call also runs
    # k_tile_y<1>, the slot-ordered copy of y, which its time leaves out)
    kern = {
        "forward": {"kernel": "k_fwd_sell<1>", "ms": fwd_ms, "min_ms": fwd_t[0],
                    "median_ms": fwd_t[len(fwd_t) // 2], "launches_timed": len(fwd_t),
                    "bytes": fwd_bytes, "GBps": fwd_bytes / fwd_ms / 1e6},
        "adjoint": {"kernel": "k_adj_csc<1>", "ms": adj_ms, "min_ms": adj_t[0],
                    "median_ms": adj_t[len(adj_t) // 2], "launches_timed": len(adj_t),
                    "bytes": adj_bytes, "GBps": adj_bytes / adj_ms / 1e6},
    }
    # the measured alternative: the atomic adjoint from the ray-major store
    # (outside the timed step; its sums depend on the order atomics land in)
    xa = torch.empty_like(x)
    atomic_ms = _time_ms(lambda: P.backproject(y, "atomic", out=xa), 20)
    atomic = {"kernel": "k_adj_atomic<1>", "ms": atomic_ms,
              "GBps_algorithmic": adj_bytes / atomic_ms / 1e6,
              "max_rel_diff_vs_deterministic":
                  float((xa - x).abs().max() / x.abs().max().clamp_min(1e-30))}
    stream = measured_stream_gbps(dev)
    copy_gbps = stream["copy_GBps"]
    dom = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom]
    from paper_2608_16960_amd.profiling import read_occupancy, read_traffic
    prof = os.path.join(ROOT, "profiles")
    for k in kern.values():
        k["traffic_bytes"] = read_traffic(os.path.join(prof, f"hbm_traffic_{w.name}.txt"),
                                          k["kernel"])
        if k["traffic_bytes"] is not None:
            k["traffic_GBps"] = k["traffic_bytes"] / k["ms"] / 1e6
    traffic = d["traffic_bytes"]
    occ = {k: read_occupancy(os.path.join(prof, "occupancy.md"), k)
           for k in ("k_fwd_sell<1>", "k_tile_y<1>", "k_adj_csc<1>", "k_otf_forward<4>",
                     "k_otf_adjoint<4, false>", "k_otf_adjoint<4, true>")}
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
                     "frac": d["GBps"] / HBM_PEAK_GBS, "traffic": traffic, "kernel": d["kernel"],
                     "timed_unit": "the kernel's own launches (every other timed step): "
                                   "HIP events the library records around it on the "
                                   "call's stream",
                     # bytes the counters saw moved, over the same time: the
                     # physical fraction (the stores hold ~5 B per segment, not 8)
                     "traffic_frac": None if traffic is None
                     else traffic / d["ms"] / 1e6 / HBM_PEAK_GBS,
                     "copy_GBps": copy_gbps, "frac_of_copy": d["GBps"] / copy_gbps,
                     "read_GBps": stream["read_GBps"],
                     "traffic_frac_of_read": None if traffic is None
                     else traffic / d["ms"] / 1e6 / stream["read_GBps"]},
        "stream": stream,
        "occupancy_waves_per_cu": occ,
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv)
                        for kk, vv in v.items()} for k, v in kern.items()},
        "atomic_adjoint": atomic,
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
    if not a.quick:
        del P
        torch.cuda.empty_cache()
        # the Large workloads last: device memory that a process has just
        # released takes the driver noticeably longer to hand out again, which
        # would show in the trace times of whatever follows them
        extras = [("tiny", "tiny workload", extra_tiny),
                  ("cnn_layers", "cnn layers", extra_cnn),
                  ("diff_csr", "differentiation workload", extra_diff_csr),
                  ("explicit_rays_medium", "explicit rays", extra_explicit_medium),
                  ("attenuated_medium", "attenuated model", extra_atten_medium),
                  ("learned_warm_start", "learned warm start", extra_learned),
                  ("onthefly_large", "large on-the-fly", extra_large_onthefly),
                  ("stored_large", "large from stored lists", extra_large_csr)]
        want = None if a.extras == "all" else set(a.extras.split(","))
        if want is not None and not want <= {k for k, _, _ in extras}:
            raise SystemExit(f"unknown extras: {sorted(want - {k for k, _, _ in extras})}")
        for key, what, fn in extras:
            if want is None or key in want:
                _log(what)
                line[key] = fn()
    if not a.no_cpu_baseline:
        _log("cpu baseline")
        line["cpu_baseline"] = cpu_baseline(w, a.cpu_views, full=a.cpu_full)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
