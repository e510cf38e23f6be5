"""Build librswr.so (HIP kernels for gfx950 + host driver) in-tree with hipcc."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "librswr.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # one IEEE operation per source operation: no contraction, no packed FP32,
    # FP32 denormals kept
    "-ffp-contract=off", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]
# the heaviest translation units first
SOURCES = ["rswr_fused_ext_f32.hip", "rswr_fused_ext_f64.hip", "rswr_fused_gen.hip",
           "rswr_adjoint_fused_f64.hip", "rswr_adjoint_fused_f32.hip", "rswr_adjoint.hip",
           "rswr_fused_plain.hip", "rswr_kernels.hip", "rswr_batch.hip",
           "rswr_fused.hip", "rswr_persist.hip", "rswr_host.cpp"]


def _compile(src, verbose):
    obj = os.path.join(CSRC, os.path.splitext(src)[0] + ".o")
    # every source is a HIP translation unit (the host driver holds the
    # device array of the no-allocation solve)
    lang = ["-x", "hip"]
    cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in res.stderr.splitlines()
                    if "is not a recognized feature" not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{err}")
    return obj, " ".join(cmd), err


def build(verbose: bool = False) -> str:
    # one hipcc per source, in parallel (the kernel files dominate)
    jobs = int(os.environ.get("MAX_JOBS", "0")) or min(len(SOURCES), os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        results = list(ex.map(lambda src: _compile(src, verbose), SOURCES))
    objs = []
    for obj, cmd, err in results:
        if verbose:
            print(cmd, flush=True)
            if err.strip():
                print(err)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
