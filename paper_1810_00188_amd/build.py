"""Build step of the HIP library: compiles csrc/rmc.hip for gfx950 into librmc.so (in-tree).

Flags: -O3, C++17, -ffp-contract=off (no implicit FMA contraction: the FP64 path keeps the
operation order of the reference algorithm; the FP32 march writes its FMAs explicitly),
packed-FP32 instructions disabled, and matrix-core instructions in their VGPR form (the
allocation network's accumulators then need no copies out of AGPRs).
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "csrc", "rmc.hip")
OUT = os.path.join(HERE, "librmc.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-mllvm", "-amdgpu-mfma-vgpr-form",
         "-I" + os.path.join(ROOT, "include"), "-I" + os.path.join(HERE, "csrc")]


def build(verbose: bool = False) -> str:
    cmd = [HIPCC] + FLAGS + [SRC, "-o", OUT + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(l for l in res.stderr.splitlines() if "packed-fp32-ops" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed ({res.returncode}):\n{errs}")
    if verbose and errs.strip():
        print(errs, file=sys.stderr)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
