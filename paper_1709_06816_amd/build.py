"""Build the HIP library libhac.so in-tree for gfx950 with hipcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhac.so")
SOURCES = [os.path.join(HERE, "csrc", f) for f in ("hac_engine.hip", "hac_rounds.hip", "hac_scan.hip", "hac_rmsd.hip", "hac_api.cpp",
                                                   "hac_serve.cpp", "hac_validate.cpp")]
HEADERS = [os.path.join(HERE, "csrc", f) for f in ("hac_engine.h", "hac_dev.h", "hac_rounds.h", "hac_ctx_info.h",
                                                   "hac_arena.h", "hac_rmsd.h", "hac_qcp.h", "hac_validate.h", "hac_scan.h")] + [
    os.path.join(ROOT, "include", "hac.h")]

# Floating point: no contraction into FMA, no fast-math, denormals kept, and no
# packed fp32 instructions (the update arithmetic must round each operation
# exactly as written).
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument", "-pthread",
]


def build(verbose: bool = False) -> str:
    """Compile every source into libhac.so (always recompiles)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-I", os.path.join(HERE, "csrc"),
           "-o", tmp, *SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in res.stdout.splitlines()
                    if "packed-fp32-ops" not in l and l.strip())
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + out)
    if verbose and out:
        print(out)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
