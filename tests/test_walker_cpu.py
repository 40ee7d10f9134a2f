"""The GPU tracer's core (boundary tables + per-ray Walker, csrc/tsp_trace_core.h)
compiled for the host with AddressSanitizer and UndefinedBehaviorSanitizer,
against the CPU FP64 oracle.

The harness (tests/walker_cpu/walk_cpu.hip) runs the same source the kernels
run, so a wrong index, a table read out of bounds or a lost crossing shows up
here without a GPU.  Bars: segment counts and voxel indices bit-exact on
every ray the oracle does not flag as a tie; FP64 lengths within 1e-10 r_max
(root conditioning: outside the flagged rays a crossing's FP64 root moves by
up to about eps |t| 1e3, and a length is the difference of two roots; the
Medium views reach 3.4e-12 r_max), 1e-7 r_max on rays the oracle marks
length-sensitive; per ray at most
2 (Nr + 1) + 2 (Ne + 1) + (Na + 1) + 2 crossing events, the row count of the
paper's padded layout (Sec. 3.3) plus the exit and the final flush.
"""
import os
import subprocess

import numpy as np
import pytest

from paper_2608_16960_amd import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "walker_cpu", "walk_cpu.hip")
EXE = os.path.join(ROOT, "_build", "walk_cpu")


@pytest.fixture(scope="session")
def walker():
    """Build the sanitised host harness (hipcc, host code only)."""
    os.makedirs(os.path.dirname(EXE), exist_ok=True)
    cmd = ["/opt/rocm/bin/hipcc", "-x", "hip", "--cuda-host-only", "-std=c++17", "-O1", "-g",
           "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2608_16960_amd", "csrc"), SRC, "-o", EXE]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        pytest.fail(f"harness build failed:\n{r.stderr[-3000:]}")
    return EXE


def _walk(exe, grid, starts, dirs, tmp_path):
    rb, eb, ab = (np.ascontiguousarray(a, np.float64) for a in grid)
    R = len(starts)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as f:
        np.array([len(rb) - 1, len(eb) - 1, len(ab) - 1], np.int32).tofile(f)
        np.array([R], np.int64).tofile(f)
        for a in (rb, eb, ab, np.ascontiguousarray(starts, np.float64),
                  np.ascontiguousarray(dirs, np.float64)):
            a.tofile(f)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(fin), str(fout)], capture_output=True, text=True, env=env)
    assert r.returncode == 0, f"walk_cpu exited {r.returncode}:\n{r.stderr[-3000:]}"
    raw = open(fout, "rb").read()
    counts = np.frombuffer(raw, np.int32, R)
    S = int(counts.sum())
    off = 4 * R
    vox = np.frombuffer(raw, np.int32, S, off)
    ln = np.frombuffer(raw, np.float64, S, off + 4 * S)
    ev = np.frombuffer(raw, np.int32, R, off + 12 * S)
    return counts, vox, ln, ev


def _compare(ora, exe, grid, starts, dirs, tmp_path, min_rays=100):
    grid = grid.arrays() if hasattr(grid, "arrays") else grid
    counts, vox, ln, ev = _walk(exe, grid, starts, dirs, tmp_path)
    tr = ora.trace(grid, starts, dirs)
    R = len(starts)
    ok = ~tr["tie"]
    assert ok.sum() >= min(min_rays, R) and ok.mean() > 0.99
    assert np.array_equal(counts[ok], tr["counts"][ok])
    mg = np.repeat(ok, counts)
    mo = np.repeat(ok, tr["counts"])
    assert np.array_equal(vox[mg], tr["vox"][mo])
    rmax = float(grid[0][-1])
    sens = np.repeat(tr["sensitive"], tr["counts"])[mo]
    tol = np.where(sens, 1e-7 * rmax, 1e-10 * rmax)
    assert np.all(np.abs(ln[mg] - tr["len"][mo]) <= tol)
    nr, ne, na = len(grid[0]) - 1, len(grid[1]) - 1, len(grid[2]) - 1
    assert ev.max() <= 2 * (nr + 1) + 2 * (ne + 1) + (na + 1) + 2
    # tie rays: the total length still agrees with the oracle's
    cg = np.concatenate([[0.0], np.cumsum(ln)])
    co = np.concatenate([[0.0], np.cumsum(tr["len"])])
    rp = np.concatenate([[0], np.cumsum(counts)])
    tg = cg[rp[1:]] - cg[rp[:-1]]
    to = co[tr["row_ptr"][1:]] - co[tr["row_ptr"][:-1]]
    assert np.all(np.abs(tg - to) <= 1e-9 * rmax)
    return int(counts.sum())


def test_tiny_views(ora, walker, tmp_path):
    w = W.tiny()
    v = w.views
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    assert _compare(ora, walker, w.grid, s, d, tmp_path) > 100000


def test_ragged_wedge_views(ora, walker, tmp_path):
    g = W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0, 9.5]),
               np.array([0.3, 0.8, 1.2, 1.5708, 2.0, 2.9]),
               np.array([-0.4, 0.3, 1.0, 1.9, 2.2, 3.0, 4.1]))
    pos = np.array([[20.0, 3.0, 5.0], [-4.0, 18.0, -7.0], [2.0, -3.0, 22.0]])
    v = W.views_at(pos, (45.0, 38.0), 37, 29, look=[0.5, -0.2, 0.1])
    s, d = ora.cone_rays(v.pos, v.look, v.up, v.fov_deg, v.H, v.W)
    _compare(ora, walker, g, s, d, tmp_path)


def test_explicit_and_degenerate_lines(ora, walker, tmp_path):
    g = W.uniform_grid((6, 8, 12), r=(1.0, 5.0))
    rng = np.random.default_rng(21)
    s, d = W.random_rays(3000, rng, r_start=(8.0, 20.0), aim=4.0)
    extra_s = np.array([[-9.0, 0.3, 0.0], [-9.0, 0.0, 0.7], [0.0, 0.0, 9.0], [6.0, 6.0, 6.0],
                        [9.0, 0.5, 0.2], [0.0, -9.0, 2.0], [7.0, 0.0, 0.0]])
    extra_d = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, -2.0], [-1.0, -1.0, -1.0],
                        [-1.0, 0.0, 0.0], [0.0, 1.0, -0.2], [-1.0, 0.0, 0.0]])
    _compare(ora, walker, g, np.concatenate([s, extra_s]), np.concatenate([d, extra_d]),
             tmp_path)


def test_interior_starts(ora, walker, tmp_path):
    for k, g in enumerate((W.uniform_grid((8, 7, 9), r=(1.0, 6.0)),
                           W.Grid(np.array([2.0, 2.7, 3.1, 4.4, 6.0]),
                                  np.array([0.3, 0.8, 1.5708, 2.9]),
                                  np.array([-0.4, 0.3, 1.9, 3.0, 4.1])))):
        rng = np.random.default_rng(60 + k)
        Ro = g.r_b[-1]
        u = rng.normal(size=(3000, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        p = u * Ro * rng.uniform(0, 1, (3000, 1)) ** (1 / 3)
        d = rng.normal(size=(3000, 3))
        p = np.concatenate([p, [[0, 0, 0], [0, 0, 0.5 * Ro], [0, 0, -0.3 * Ro]]])
        d = np.concatenate([d, [[0.3, 0.4, 0.5], [1.0, 0.2, -0.1], [-0.5, 0.1, 0.3]]])
        (tmp_path / str(k)).mkdir()
        _compare(ora, walker, g, p, d, tmp_path / str(k))


def test_parallel_views(ora, walker, tmp_path):
    from oracle.views import parallel_rays
    g = W.uniform_grid((7, 9, 11), r=(0.5, 4.0))
    s, d = parallel_rays([[9.0, 2.0, -1.0], [-3.0, 0.0, 9.5]], [[0, 0, 0], [0.2, 0.1, 0]],
                         [0, 0, 0], (8.5, 8.5), 40, 40)
    _compare(ora, walker, g, s, d, tmp_path)


def test_medium_two_views(ora, walker, tmp_path):
    """Two of the Medium workload's 30 views (131,072 rays, 50^3 grid)."""
    w = W.medium()
    v = w.views
    sel = [0, 17]
    s, d = ora.cone_rays(v.pos[sel], v.look[sel], v.up[sel], v.fov_deg[sel], v.H, v.W)
    assert _compare(ora, walker, w.grid, s, d, tmp_path) > 10_000_000
