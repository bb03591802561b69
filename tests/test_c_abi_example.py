"""The library through its C-ABI alone: a plain C program (tests/c_abi_example.c)
compiled against include/odust.h and libodust.so, with no Python in the
path.  On the CPU the program must compile and link warning-free; on the GPU
it runs the small single-grain configuration and checks its own results."""
import os
import subprocess

import pytest

from paper_2205_06557_amd import build as Bld


def test_c_example_compiles_and_links(tmp_path):
    if not os.path.exists(Bld.LIB):
        pytest.fail("libodust.so is not built")
    out = str(tmp_path / "c_abi_example")
    subprocess.run(Bld.c_example_command(out), check=True, capture_output=True, text=True)
    assert os.path.exists(out)


@pytest.mark.gpu
def test_c_example_runs():
    assert os.path.exists(Bld.C_EXAMPLE), "tests/c_abi_example is not built (run build())"
    r = subprocess.run([Bld.C_EXAMPLE], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    assert "charge" in r.stdout
