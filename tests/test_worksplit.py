"""The host-side work split of the symmetric all-pairs sum takes every
unordered pair of 256-ion tiles exactly once, for 1..700 tiles and a few
large counts, in both the grouped-rows and single-row forms (a plain C++
check of csrc/worksplit.hpp, compiled here with g++ under AddressSanitizer
and UBSan; no GPU)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2205_06557_amd", "csrc")


def test_every_tile_pair_once(tmp_path):
    exe = str(tmp_path / "worksplit_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Werror", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-I", CSRC,
                    os.path.join(HERE, "worksplit_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "grouped rows" in r.stdout
