"""Kernels whose items can outnumber one dispatch (elementwise passes over
4V or B*V items, one wavefront per voxel) stride over grids capped at 2^23
workgroups.  Here a child process runs tests/strided_case.py with the cap
lowered to 3 workgroups (TSP_MAX_BLOCKS), so that each thread or wavefront
takes many items, and its results must equal this process's at the default
cap: bitwise for the forward, the deterministic and fixed-point adjoints and
the vector kernels (their arithmetic does not depend on which thread takes
an item); within 1e-5 of the absolute sums for the atomic adjoints, whose
order of addition does.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def test_capped_grids_give_the_same_results(tmp_path):
    sys.path.insert(0, HERE)
    import strided_case
    ref = strided_case.compute()
    out = tmp_path / "capped.npz"
    env = dict(os.environ, TSP_MAX_BLOCKS="3")
    print("child: strided_case.py with TSP_MAX_BLOCKS=3", flush=True)
    r = subprocess.run([sys.executable, os.path.join(HERE, "strided_case.py"), str(out)], env=env,
                       capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-3000:]
    got = np.load(out)
    assert sorted(got.files) == sorted(ref)
    for k, v in ref.items():
        if "atomic" in k:
            scale = np.abs(v).max()
            assert np.all(np.abs(got[k] - v) <= 1e-5 * scale), k
        else:
            assert np.array_equal(got[k], v), k
