"""Build the C-ABI caller (tests/c_caller/lbm_c_caller) against the in-tree
liblbm.so: a test program that uses include/lbm.h and the HIP runtime only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "lbm_c_caller.cpp")
BIN = os.path.join(HERE, "lbm_c_caller")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(verbose: bool = False) -> str:
    lib_dir = os.path.join(ROOT, "paper_1803_07822_amd")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17", "-Wall",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-I", os.path.join(ROOT, "include"), SRC, "-o", BIN + ".tmp",
           "-L", lib_dir, "-llbm", "-Wl,-rpath,$ORIGIN/../../paper_1803_07822_amd"]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"building the C-ABI caller failed:\n{r.stdout}\n{r.stderr}")
    os.replace(BIN + ".tmp", BIN)
    return BIN


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
