"""The work lists (csrc/wmi_plan.h) on random inputs, on the CPU: coverage
and the capacity limits the main kernel's LDS layout relies on, for batches
and for serving launches."""
import os
import subprocess
import tempfile

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plan_invariants():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "plan_check")
        subprocess.run(["g++", "-O1", "-std=c++17", "-Wall", "-Werror",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-I", os.path.join(ROOT, "paper_2204_09131_amd", "csrc"),
                        os.path.join(ROOT, "tests", "plan_check.cpp"), "-o", exe], check=True)
        r = subprocess.run([exe, "400"], capture_output=True, text=True, timeout=300)
        assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
