"""The oracle under AddressSanitizer and UndefinedBehaviorSanitizer, on the
CPU: oracle.c is compiled with gcc into a small driver
(oracle_check.c) that runs every entry point on adversarial inputs with
exactly sized buffers and capacities below the counts."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-Wall", "-Werror", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "oracle"), os.path.join(HERE, "oracle_check.c"),
           os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert int(r.stdout.split()[1]) > 100000  # checks that ran
