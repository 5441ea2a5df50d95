"""Host checks of the tile-walk planning (no GPU).

Builds the planner (paper_2208_10978_amd/csrc/plan.cpp) with the host C++
compiler next to tests/plan_check.cpp and runs it: every rotation walk
(forward, per-parameter and per-string reverse schedules of a seeded
Jordan-Wigner-shaped UCCSD list) and every fast record of a seeded Pauli-sum
tiling must split its free bits into lane and loop bits, visit each free-bit
pattern once, carry the right LDS slots and parity lanes, and reach the least
bank-conflict cost over all choices of lane bits."""
import pathlib
import shutil
import subprocess

import pytest

ROOT = pathlib.Path(__file__).resolve().parents[1]
CSRC = ROOT / "paper_2208_10978_amd" / "csrc"


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_tile_walks(tmp_path):
    exe = tmp_path / "plan_check"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", str(CSRC), str(ROOT / "tests" / "plan_check.cpp"),
                    str(CSRC / "plan.cpp"), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok "), out.stdout
