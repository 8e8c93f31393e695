"""The C ABI from a plain C99 program: one anneal on the GPU (NULL stream),
checked inside the program against the C oracle element by element."""
import os
import shutil
import subprocess

import pytest

from tests.conftest import ROOT, load_binding

pytestmark = pytest.mark.gpu
load_binding()  # fails loudly when the library is missing


def test_c_program_anneal_equals_oracle(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    pkg = os.path.join(ROOT, "paper_2311_09275_amd")
    orc = os.path.join(ROOT, "oracle")
    exe = str(tmp_path / "gpu_anneal")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(ROOT, "include"), "-I", orc,
                    os.path.join(ROOT, "tests", "c", "gpu_anneal.c"),
                    "-L", pkg, "-lising", "-L", orc, "-loracle",
                    f"-Wl,-rpath,{pkg}", f"-Wl,-rpath,{orc}", "-o", exe], check=True)
    print("running", exe, flush=True)
    out = subprocess.run([exe], capture_output=True, text=True, timeout=90)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "ok"
