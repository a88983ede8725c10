"""Host logic on the CPU: the planner's op lists (products, batches,
truncated transforms, BasisCvt passes, products with 128-bit words over
TGF(2^256), the simple variant of Alg. 4, the Frobenius-partition variant of
App. C, BasisCvt sub-conversions run inside FFT passes) executed sequentially with the same
tile bodies the kernels run, compared with the oracle; the kernels' block to
tile order visits every tile once (no GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1708_09746_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
ROCM_INC = "/opt/rocm/include"


@pytest.fixture(scope="module")
def host_exec(tmp_path_factory):
    if not os.path.exists(HIPCC) or shutil.which("gcc") is None:
        pytest.skip("needs hipcc and gcc")
    d = tmp_path_factory.mktemp("host_exec")
    orc = d / "oracle.o"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-pthread", "-c",
                    os.path.join(ROOT, "oracle", "gf2x_oracle.c"), "-o", str(orc)], check=True)
    obj = d / "check.o"
    # host-only compile of the kernel headers (no device code in this file)
    subprocess.run([HIPCC, "-O2", "-std=c++17", "-fPIC", "-I", ROCM_INC, "-I", CSRC, "-c",
                    os.path.join(ROOT, "tests", "cpp", "host_exec_check.cpp"), "-o", str(obj)], check=True)
    exe = d / "host_exec_check"
    subprocess.run(["g++", str(obj), str(orc), "-o", str(exe), "-pthread", "-L/opt/rocm/lib", "-lamdhip64",
                    "-Wl,-rpath,/opt/rocm/lib"], check=True)
    return str(exe)


@pytest.mark.parametrize("what", ["products", "batch", "trunc", "basiscvt", "xcd", "w128", "simple", "frobenius",
                                  "fusion"])
def test_host_execution_matches_oracle(host_exec, what):
    out = subprocess.run([host_exec, what], capture_output=True, text=True, timeout=600)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "host exec ok" in out.stdout
