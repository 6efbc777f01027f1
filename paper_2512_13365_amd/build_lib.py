"""Build libcse.so, the gfx950 HIP library behind include/cse.h.

Compiles the single translation unit csrc/cse_api.hip with hipcc for gfx950
into paper_2512_13365_amd/libcse.so (in-tree, next to the binding).
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "cse_api.hip")
LIB = os.path.join(HERE, "libcse.so")
# VALU / LDS microbenchmarks read by bench.py --calibrate (not part of the ABI).
CALIB_SRC = os.path.join(HERE, "csrc", "cse_calib.hip")
CALIB_LIB = os.path.join(HERE, "libcse_calib.so")
ARCH = os.environ.get("CSE_OFFLOAD_ARCH", "gfx950")


def hipcc_cmd(out: str, extra=(), src: str = SRC):
    return ["hipcc", "-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
            *extra, "-o", out, src]


def build(verbose: bool = False) -> str:
    cmd = hipcc_cmd(LIB + ".tmp")
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = hipcc_cmd(CALIB_LIB + ".tmp", src=CALIB_SRC)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CALIB_LIB + ".tmp", CALIB_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
