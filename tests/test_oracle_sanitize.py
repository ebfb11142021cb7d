"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
tests/oracle_sanitize_driver.c runs every oracle entry point (the find in
its plain, material, field and steering variants, the parity prefixes and
path check, backward fit, smoothing, fit, triplet seeding, duplicate
removal, seed cleaning and the network) on a small deterministic event, in
a gcc build with both sanitizers; any report fails the test.  CPU only."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_is_clean_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-std=c99", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-o", exe, os.path.join(HERE, "oracle_sanitize_driver.c"),
           os.path.join(ROOT, "oracle", "mkf_oracle.c"), os.path.join(ROOT, "oracle", "mkf_mlp.c"),
           "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr
    assert "oracle driver ok" in res.stdout
