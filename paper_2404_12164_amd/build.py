"""Build the HIP library libfte.so in-tree for gfx950 with hipcc."""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libfte.so")
SOURCES = ["fte_api.hip", "fte_kernels.hip"]
HEADERS = ["fte_internal.hpp", "fte_device.hpp"]


def hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose: bool = False, defines=(), out: str = None) -> str:
    """Compile every source (always; the caller asked for a build).
    ``defines`` are extra -D macros (tuning knobs of fte_internal.hpp and the
    step kernel); ``out`` another path for the library."""
    lib = out or LIB
    objs = []
    # -ffp-contract=on: a fused multiply-add only where one source expression
    # has the a * b + c shape, decided by the front end; the default (fast)
    # lets the back end fuse a product into a sum of another statement when
    # both land in one basic block, so that the same arithmetic could round
    # differently in two kernel instances whose branches differ
    common = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Wall", "-Wno-unused-result",
              "-ffp-contract=on",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-munsafe-fp-atomics",
              "-I", os.path.join(HERE, "..", "include")]
    for src in SOURCES:
        obj = lib + "." + src.replace(".hip", ".o")
        cmd = [hipcc()] + common + [f"-D{d}" for d in defines] + ["-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = lib + ".tmp"
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    for o in objs:
        os.remove(o)
    return lib


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
