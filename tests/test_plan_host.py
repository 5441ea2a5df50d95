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


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_tile_walks_under_host_sanitizers(tmp_path):
    """The same checks with AddressSanitizer and UndefinedBehaviorSanitizer
    on the planner (host code only): out-of-bounds accesses, use after free,
    shifts past the width and signed overflow abort the run."""
    probe = subprocess.run(["g++", "-fsanitize=address,undefined", "-x", "c++", "-", "-o", str(tmp_path / "p")],
                           input="int main(){return 0;}", capture_output=True, text=True)
    if probe.returncode != 0:
        pytest.skip("host sanitizer runtime not available")
    exe = tmp_path / "plan_check_san"
    subprocess.run(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-std=c++17", "-I", str(CSRC), str(ROOT / "tests" / "plan_check.cpp"),
                    str(CSRC / "plan.cpp"), "-o", str(exe)], check=True)
    env = {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0", "UBSAN_OPTIONS": "print_stacktrace=1"}
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout[-2000:] + out.stderr[-4000:]
    assert out.stdout.startswith("ok "), out.stdout
