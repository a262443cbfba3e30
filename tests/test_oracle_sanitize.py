"""The oracle under the sanitizers.

The oracle's C source is linked with a driver (tests/sanitize/oracle_exercise.c)
that calls every entry point on seeded inputs spanning the edge cases, on one
worker thread and on the block pool, and requires the expected status codes,
sorted sort outputs and byte-identical results for both thread counts.  It is
built twice with gcc as standalone executables: with AddressSanitizer +
UndefinedBehaviorSanitizer (out-of-bounds accesses, use after free, leaks,
signed overflow, bad shifts and conversions abort the run), and with
ThreadSanitizer for the block-parallel mode (a data race between blocks of
the pool aborts the run).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = [os.path.join(ROOT, "oracle", "coxo.c"), os.path.join(ROOT, "tests", "sanitize", "oracle_exercise.c")]
COMMON = ["-std=gnu11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fno-fast-math",
          "-fno-strict-aliasing", "-pthread", "-Wall", "-Wno-unused-function"]
BUILDS = {
    "asan_ubsan": ["-fsanitize=address,undefined", "-fno-sanitize-recover=all"],
    "tsan": ["-fsanitize=thread"],
}
ENV = {
    "asan_ubsan": {"ASAN_OPTIONS": "abort_on_error=0:halt_on_error=1:exitcode=65",
                   "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"},
    "tsan": {"TSAN_OPTIONS": "halt_on_error=1:exitcode=66"},
}


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.skipif(bool(os.environ.get("LD_PRELOAD")), reason="a preloaded library keeps the sanitizer runtimes "
                    "from loading first")
@pytest.mark.parametrize("kind", sorted(BUILDS))
def test_oracle_is_clean_under_sanitizer(kind, tmp_path):
    exe = str(tmp_path / f"oracle_exercise_{kind}")
    b = subprocess.run(["gcc", *COMMON, *BUILDS[kind], *SRC, "-o", exe, "-lm"], capture_output=True, text=True)
    if b.returncode != 0 and "cannot find" in b.stderr and "san" in b.stderr:
        pytest.skip(f"sanitizer runtime for {kind} not installed")
    assert b.returncode == 0, b.stderr
    env = dict(os.environ, **ENV[kind])
    r = subprocess.run([exe, "8"], capture_output=True, text=True, env=env, timeout=900)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    assert r.stdout.startswith("ok ")
    assert "WARNING" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-6000:]
