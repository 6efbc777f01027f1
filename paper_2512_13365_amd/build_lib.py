"""Build libcse.so, the gfx950 HIP library behind include/cse.h.

The host runtime (csrc/cse_api.hip) and the step kernels of each row-word
count (csrc/cse_step.hip compiled once per W = 1..8) are separate
translation units, compiled in parallel with hipcc for gfx950 and linked
into paper_2512_13365_amd/libcse.so (in-tree, next to the binding).  The
VALU / LDS microbenchmarks (csrc/cse_calib.hip) become libcse_calib.so.
"""
import os
import subprocess
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
SRC = os.path.join(CSRC, "cse_api.hip")
STEP_SRC = os.path.join(CSRC, "cse_step.hip")
LIB = os.path.join(HERE, "libcse.so")
# VALU / LDS microbenchmarks read by bench.py --calibrate (not part of the ABI).
CALIB_SRC = os.path.join(CSRC, "cse_calib.hip")
CALIB_LIB = os.path.join(HERE, "libcse_calib.so")
ARCH = os.environ.get("CSE_OFFLOAD_ARCH", "gfx950")
ROW_WORDS = range(1, 9)


def _flags():
    return ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wall", "-Wno-unused-function",
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def hipcc_cmd(out: str, extra=(), src: str = SRC):
    """One-step build of a single-source shared library."""
    return ["hipcc", *_flags(), "-shared", *extra, "-o", out, src]


def _run_parallel(cmds, verbose, jobs):
    running, i = [], 0
    while i < len(cmds) or running:
        while i < len(cmds) and len(running) < jobs:
            if verbose:
                print(" ".join(cmds[i]), flush=True)
            running.append((cmds[i], subprocess.Popen(cmds[i])))
            i += 1
        cmd, p = running.pop(0)
        if p.wait() != 0:
            for _, q in running:
                q.wait()
            raise subprocess.CalledProcessError(p.returncode, cmd)


def build(verbose: bool = False) -> str:
    jobs = max(1, min(int(os.environ.get("MAX_JOBS", os.cpu_count() or 1)), 16))
    with tempfile.TemporaryDirectory(prefix="cse_build_") as tmp:
        objs = [os.path.join(tmp, "cse_api.o")]
        cmds = [["hipcc", *_flags(), "-c", "-o", objs[0], SRC]]
        for w in ROW_WORDS:
            o = os.path.join(tmp, f"cse_step_w{w}.o")
            objs.append(o)
            cmds.append(["hipcc", *_flags(), f"-DCSE_STEP_W={w}", "-c", "-o", o, STEP_SRC])
        _run_parallel(cmds, verbose, jobs)
        link = ["hipcc", f"--offload-arch={ARCH}", "-fPIC", "-shared", "-o", LIB + ".tmp", *objs]
        if verbose:
            print(" ".join(link), flush=True)
        subprocess.run(link, check=True)
    os.replace(LIB + ".tmp", LIB)
    cmd = hipcc_cmd(CALIB_LIB + ".tmp", src=CALIB_SRC)
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(CALIB_LIB + ".tmp", CALIB_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
