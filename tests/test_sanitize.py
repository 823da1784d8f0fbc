"""The C code of the oracle and of the input generator, built with gcc's
AddressSanitizer and UndefinedBehaviorSanitizer and run through
tests/sanitize_driver.c: its pins (the worked example, the metric axioms, the
k = 1 closed form, degree sums, row/query agreement, the network analyses)
must pass with no sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SOURCES = [os.path.join(ROOT, "tests", "sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "oracle", "k1.c"),
           os.path.join(ROOT, "oracle", "graph.c"),
           os.path.join(ROOT, "synth", "gen.c")]


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(tmp_path_factory.mktemp("san") / "sanitize_driver")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", *SOURCES, "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_oracle_and_generator_are_clean_under_asan_and_ubsan(driver):
    env = dict(os.environ)
    env["OMP_NUM_THREADS"] = "2"
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([driver], capture_output=True, text=True, env=env, timeout=300)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report
    assert "runtime error" not in report and "AddressSanitizer" not in report, report
    assert "all checks passed" in r.stdout
