"""Build the HIP library libgbp_hip.so in-tree for gfx950.

Both translation units go through hipcc. Packed FP32 instructions are
disabled for device code (the flag only matters for the device pass; the
host pass warns that it does not know the feature)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libgbp_hip.so")
ARCH = os.environ.get("GBP_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-ffp-contract=fast", "-Wall", "-Wno-unused-parameter",
             "-Wno-unused-variable", "-Wno-unused-command-line-argument"]


def build(verbose: bool = False) -> str:
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for src in ("gbp_kernels.hip", "gbp_mlp.hip", "gbp_api.cpp"):
        obj = os.path.join(HERE, "_build", src + ".o")
        cmd = ["hipcc", "-c", *HIP_FLAGS]
        if src.endswith(".cpp"):
            cmd += ["-x", "hip"]
        cmd += [os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = OUT + ".tmp"
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), file=sys.stderr)
    subprocess.run(cmd, check=True)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
