"""The oracle's CPU pins, run again on an AddressSanitizer + UndefinedBehavior
Sanitizer build of oracle.c: an out-of-bounds access, a use of freed memory,
a signed overflow or a misaligned access anywhere in the paths the pins
exercise aborts the run.  CPU only (the GPU library is not involved)."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# the suites that call the oracle (the Philox test builds rocRAND with hipcc
# and the planted-mistake test runs gcc: neither runs under the preload)
SUITES = ["tests/test_oracle_pins.py", "tests/test_oracle_pins_material.py", "tests/test_oracle_frame.py",
          "tests/test_oracle_lobes.py", "tests/test_oracle_vpl.py"]


def _runtime(name):
    r = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = r.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_asan_ubsan():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (asan and ubsan):
        pytest.skip("sanitizer runtimes not installed")
    from oracle import build as obuild
    with tempfile.TemporaryDirectory() as d:
        so = obuild.build(out=os.path.join(d, "liboracle_san.so"), sanitize=True)
        # reports go to files: pytest's capture would swallow them when the
        # sanitizer ends the process
        logs = os.path.join(d, "san")
        env = dict(os.environ, PG_ORACLE_LIB=so, LD_PRELOAD=f"{asan} {ubsan}",
                   ASAN_OPTIONS=f"detect_leaks=0:log_path={logs}",
                   UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={logs}")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            "-k", "not rocrand and not planted", *SUITES],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=1500)
        reports = "".join(open(os.path.join(d, f)).read() for f in sorted(os.listdir(d)) if f.startswith("san"))
    tail = (reports[:3000] + r.stdout[-2000:] + r.stderr[-1000:])
    assert r.returncode == 0 and not reports, tail
    assert "passed" in r.stdout and "failed" not in r.stdout, tail
