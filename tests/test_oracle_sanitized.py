"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code; no GPU): oracle/sanitize_check.c runs every oracle routine -- brick
assembly in both problems and all orders, DG, Stokes blocks, simplices,
Nedelec and Raviart-Thomas, numbering, patterns, PCG, L2 errors -- with
leak detection on, and checks a few exact properties on the way.  A second
case confirms the sanitizer build does catch a planted heap overflow, so a
clean run means something."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")
FLAGS = ["-std=c99", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer"]

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")


def _build_and_run(src_path, out_dir, extra=()):
    exe = os.path.join(out_dir, "a.out")
    subprocess.run(["gcc", *FLAGS, *extra, "-I", ORACLE, "-o", exe, src_path, "-lm"], check=True,
                   capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    return subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)


def test_oracle_runs_clean_under_address_and_undefined_sanitizers():
    with tempfile.TemporaryDirectory() as td:
        r = _build_and_run(os.path.join(ORACLE, "sanitize_check.c"), td)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "all checks passed" in r.stdout


def test_sanitizer_build_catches_a_planted_overflow():
    src = "#include <stdlib.h>\nint main(void){int *a = malloc(4 * sizeof(int)); a[4] = 1; free(a); return 0;}\n"
    with tempfile.TemporaryDirectory() as td:
        p = os.path.join(td, "bad.c")
        with open(p, "w") as f:
            f.write(src)
        r = _build_and_run(p, td)
    # reported by AddressSanitizer, or first by UBSan's object-size check
    assert r.returncode != 0
    assert "heap-buffer-overflow" in r.stderr or "insufficient space" in r.stderr, r.stderr[-2000:]
