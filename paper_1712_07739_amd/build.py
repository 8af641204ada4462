"""Build libdfmm.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdfmm.so")
SOURCES = ["api.hip", "setup.hip", "tree.hip", "adaptive.hip", "fmm.hip", "mlp.hip", "batch.hip"]
PROBE = "probe_lds_passes.hip"
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-value", "-Wno-unused-result",
    "-I" + os.path.join(HERE, "..", "include"),
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    bdir = os.path.join(HERE, "_build")
    os.makedirs(bdir, exist_ok=True)

    def compile_one(src):
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [hipcc, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        return obj

    def probe():
        # the LDS pass probe behind the M2L kernels' lane map: a program of
        # its own, not part of the library
        cmd = [hipcc, *FLAGS, os.path.join(CSRC, PROBE), "-o", os.path.join(bdir, PROBE.replace(".hip", ""))]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=len(SOURCES) + 1) as ex:
        fp = ex.submit(probe)
        objs = list(ex.map(compile_one, SOURCES))
        fp.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
