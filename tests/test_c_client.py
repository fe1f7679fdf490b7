"""The C ABI from plain C: tests/c_client/client.c includes only
include/ht.h and the HIP runtime API, links libht.so, and checks its own
results.  Compiling and linking needs no GPU; running it does."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1712_09494_amd")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build_client(out):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    if not os.path.exists(os.path.join(PKG, "libht.so")):
        pytest.skip("libht.so not built")
    cmd = ["gcc", "-std=c11", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           f"-I{ROCM}/include", f"-I{ROOT}/include", os.path.join(ROOT, "tests", "c_client", "client.c"),
           "-o", out, f"-L{PKG}", "-lht", f"-L{ROCM}/lib", "-lamdhip64",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return out


def test_c_client_compiles_and_links(tmp_path):
    build_client(str(tmp_path / "client"))


@pytest.mark.gpu
def test_c_client_runs(tmp_path):
    exe = build_client(str(tmp_path / "client"))
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.count(" ok") == 6, r.stdout
