"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

The real-valued source is compiled twice (double and float).  Floating-point
contraction and fast-math are off and no FTZ/DAZ mode is set, so every fma in
the source is the only fused operation.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

CFLAGS = ["-O2", "-march=x86-64-v3", "-std=c11", "-fPIC", "-ffp-contract=off", "-fno-fast-math",
          "-fopenmp", "-Wall", "-Wno-unknown-pragmas"]


def build(verbose: bool = False) -> str:
    objs = []
    units = [("rswr_layout.c", []),
             ("rswr_oracle_real.c", []),
             ("rswr_oracle_real.c", ["-DORACLE_F32"])]
    for i, (src, extra) in enumerate(units):
        obj = os.path.join(HERE, f"_oracle_{i}.o")
        cmd = ["gcc", *CFLAGS, *extra, "-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd))
        subprocess.check_call(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = ["gcc", "-shared", "-fopenmp", "-o", tmp, *objs, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
