"""Computes a fixed set of projector and vector results on cuda:0 and saves
them to an .npz (argv[1]).  tests/test_gpu_strided.py runs it in a child
process with TSP_MAX_BLOCKS set to a tiny launch cap, so that every kernel
that strides over capped grids takes many items per thread or wavefront, and
compares the results with the same computation in its own process.
"""
import os
import sys

import numpy as np
import torch

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from paper_2608_16960_amd import nn as NN  # noqa: E402
from paper_2608_16960_amd import workloads as W  # noqa: E402
from paper_2608_16960_amd.projector import Projector  # noqa: E402


def compute():
    dev = torch.device("cuda", 0)
    w = W.tiny()
    rng = np.random.default_rng(90)
    out = {}
    rho = torch.from_numpy(rng.uniform(0, 1, (5, *w.grid.shape)).astype(np.float32)).to(dev)
    for mode in ("csr", "onthefly"):
        P = Projector(w.grid, views=w.views, mode=mode)
        yy = torch.from_numpy(rng.normal(size=(5, *P.out_shape)).astype(np.float32)).to(dev)
        out[f"{mode}_fwd"] = P.forward(rho).cpu().numpy()
        for m in ("deterministic", "atomic") + (("fixedpoint",) if mode == "onthefly" else ()):
            out[f"{mode}_{m}"] = P.backproject(yy, m).cpu().numpy()
        P.close()
    g = W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0, 9.5]), np.array([0.3, 0.8, 1.2, 1.5708, 2.0, 2.9]),
               np.array([-0.4, 0.3, 1.0, 1.9, 2.2, 3.0, 4.1]))
    s, d = W.random_rays(1500, np.random.default_rng(91), r_start=(12.0, 20.0), aim=5.0)
    P = Projector(g, rays=(s, d))
    yy = torch.from_numpy(rng.normal(size=(3, *P.out_shape)).astype(np.float32)).to(dev)
    out["wedge_deterministic"] = P.backproject(yy, "deterministic").cpu().numpy()
    P.close()
    a = torch.from_numpy(rng.normal(size=(3, 70000)).astype(np.float32)).to(dev)
    x = torch.from_numpy(rng.normal(size=(3, 70000)).astype(np.float32)).to(dev)
    out["axpy"] = NN.axpy(x.clone(), a, 0.75).cpu().numpy()
    out["scale"] = NN.scale(a, -1.5).cpu().numpy()
    out["bf16"] = NN.from_bf16(NN.to_bf16(a)).cpu().numpy()
    p = x.clone()
    opt = NN.Adam([p], lr=1e-2)
    for _ in range(3):
        opt.step([a])
    out["adam"] = p.cpu().numpy()
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    np.savez(sys.argv[1], **compute())
    print("saved", sys.argv[1], flush=True)
