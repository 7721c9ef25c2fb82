"""Host-side layout checks on the CPU: the hybrid Gauss-Seidel schedule
(depths, in-block entry ranges, 1 / a_ii) and the row tiles with column
dictionaries of rectangular matrices (the smoothed prolongator's P and P^T),
each against a brute-force scan on random matrices.  The checker
(tests/cpp/host_layout_check.cpp) is compiled here with the host setup source
(csrc/setup.cpp, the same flags as the library build)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_gauss_seidel_schedule_and_row_tiles(tmp_path):
    exe = str(tmp_path / "host_layout_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-pthread", "-ffp-contract=off", "-fno-fast-math",
                    "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2210_16660_amd", "csrc"),
                    os.path.join(ROOT, "tests", "cpp", "host_layout_check.cpp"),
                    os.path.join(ROOT, "paper_2210_16660_amd", "csrc", "setup.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("0 failures")
