"""CPU tests of the library's host-side logic (no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_hole_fixup_planner(tmp_path):
    exe = tmp_path / "test_holes"
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-fsanitize=address,undefined",
                           "-I", os.path.join(ROOT, "paper_2203_04774_amd", "csrc"),
                           "-o", str(exe), os.path.join(ROOT, "tests", "cpp", "test_holes.cpp")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout + out.stderr
