"""The oracle's own pins, re-run against a build of the oracle with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only): every
array access of the C oracle on those inputs is bounds-checked, and signed
overflow, bad shifts and the like abort the run."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_pins_under_sanitizers(tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    lib = ob.build_sanitized(str(tmp_path / "liboracle_asan.so"))
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    env = dict(os.environ, TSP_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="4")
    tests = [os.path.join(HERE, f) for f in ("test_oracle_pins.py", "test_oracle_cone_rays.py",
                                              "test_oracle_views.py", "test_oracle_interior.py",
                                              "test_oracle_dynamic.py", "test_oracle_atten.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        *tests], capture_output=True, text=True, env=env, cwd=ROOT, timeout=900)
    assert r.returncode == 0, (r.stdout[-3000:] + r.stderr[-3000:])
    assert "passed" in r.stdout
