"""The oracle and the input generators built with AddressSanitizer and
UndefinedBehaviorSanitizer (gcc, host code only) and run on small graphs of
every generator: out-of-bounds accesses, leaks and undefined behaviour in
the checker or the generators fail here.  The driver
(`tests/sanitize_host.c`) also checks invariants that hold for any input
(forest size = n - components, identity multilinear = smallest incident key,
no edge between component stars)."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_and_generators_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path / "sanitize_host")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(ROOT, "tests", "sanitize_host.c"),
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "gen", "gen.c"), "-lm", "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr
    env = dict(os.environ)
    # a library preloaded by the environment would come before the
    # sanitizer runtime; the check of that order is switched off, nothing
    # else about the environment changes
    env["ASAN_OPTIONS"] = "detect_leaks=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1"
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, run.stdout + run.stderr
    assert run.stdout.strip().endswith("ok"), run.stdout
