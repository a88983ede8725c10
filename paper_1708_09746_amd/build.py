"""Build libgf2x_afft.so (HIP, gfx950) in the package directory."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libgf2x_afft.so")
SOURCES = [os.path.join(HERE, "csrc", "afft.hip")]
ARCH = os.environ.get("GF2X_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out):
    return [
        "/opt/rocm/bin/hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        "-Wall", "-Wno-unused-function",
        # packed FP32 ops are kept out of the device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        "-o", out,
    ] + SOURCES


def build() -> str:
    tmp = LIB + ".tmp"
    subprocess.check_call(hipcc_cmd(tmp))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
