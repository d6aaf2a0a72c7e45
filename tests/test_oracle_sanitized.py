"""The oracle built with the address and undefined-behaviour sanitizers
(tests/cpu/oracle_check.cpp includes its source): both curves, both metrics
and three dimensions against brute force on adversarial inputs, so that an
access outside an array or an undefined shift anywhere in the oracle aborts
the run rather than passing unnoticed."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call([
        "g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
        "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-ffp-contract=off",
        "-pthread", os.path.join(ROOT, "tests", "cpu", "oracle_check.cpp"), "-o", exe])
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr[-3000:]
    assert r.stdout.strip() == "ok"
