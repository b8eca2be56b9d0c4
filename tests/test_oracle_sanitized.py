"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer: the C
source is rebuilt with both (host code, gcc, every report fatal) and the
oracle pins run against that build in a child process.  Any out-of-bounds
access, use after free, leak-free misuse or undefined arithmetic in the
oracle fails the run."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PINS = ["test_oracle_knn.py", "test_oracle_normals.py", "test_oracle_icp.py", "test_oracle_metrics.py",
        "test_oracle_projective.py", "test_oracle_radius.py"]


def _asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if r.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_sanitizers(tmp_path):
    import oracle
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's ASan runtime is not installed")
    lib = oracle.build_sanitized(str(tmp_path / "_oracle_san.so"))
    env = dict(os.environ, ORACLE_LIB=lib, LD_PRELOAD=rt,
               # the interpreter itself is not instrumented: leaks at exit are
               # its own; every oracle report stops the run
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    # the child loads the sanitized build, not the plain one
    chk = subprocess.run([sys.executable, "-c", "import oracle; print(oracle._load()._name)"], cwd=ROOT, env=env,
                         capture_output=True, text=True, timeout=120)
    assert chk.returncode == 0 and chk.stdout.strip() == lib, chk.stdout + chk.stderr
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        *[os.path.join(ROOT, "tests", p) for p in PINS]],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
