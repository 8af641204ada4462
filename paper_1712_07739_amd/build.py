"""Build libdfmm.so (HIP, gfx950) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdfmm.so")
SOURCES = ["api.hip", "setup.hip", "tree.hip", "adaptive.hip", "fmm.hip", "mlp.hip", "batch.hip"]
PROBES = ["probe_lds_passes.hip", "probe_valu_rates.hip"]
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

    def probe(src):
        # the measurement programs behind the M2L kernels' lane map and the
        # VALU rooflines: programs of their own, not part of the library
        cmd = [hipcc, *FLAGS, os.path.join(CSRC, src), "-o", os.path.join(bdir, src.replace(".hip", ""))]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)

    with ThreadPoolExecutor(max_workers=len(SOURCES) + len(PROBES)) as ex:
        fps = [ex.submit(probe, src) for src in PROBES]
        objs = list(ex.map(compile_one, SOURCES))
        for fp in fps:
            fp.result()
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-o", tmp, *objs], check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
