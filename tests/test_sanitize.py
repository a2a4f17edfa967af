"""Sanitizer build on the CPU: every oracle entry point, under
AddressSanitizer (with leak detection) and UndefinedBehaviorSanitizer, on
small seeded instances with the grid stencil, explicit predecessor lists and
the objective variants (oracle/sanitize_check.c)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _have_asan():
    r = subprocess.run(["gcc", "-fsanitize=address", "-x", "c", "-", "-o", os.devnull],
                       input="int main(void){return 0;}", capture_output=True, text=True)
    return r.returncode == 0


@pytest.mark.skipif(not _have_asan(), reason="gcc without AddressSanitizer")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = tmp_path / "oracle_asan"
    src = os.path.join(ROOT, "oracle")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", src, os.path.join(src, "oracle.c"), os.path.join(src, "sanitize_check.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("ok"), r.stdout
    assert "runtime error" not in r.stderr, r.stderr
