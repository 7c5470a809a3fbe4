"""Build the CPU oracle shared libraries (test infrastructure only).

Three builds of lbm_oracle.c:
  liboracle_f64.so    REAL = double  (the FP64 reference, operation-order twin)
  liboracle_f32.so    REAL = float   (emulation of the reduced-precision storage modes)
  liboracle_plain.so  REAL = double, PLAIN  (the textbook operation order: plain sums
                      over all populations, plain inverse-transform rows, no fma)

Flags: -O2 -ffp-contract=off (no fused multiply-add the source does not write, so
every product and sum is rounded as written; the SMRT moment transforms call fma
explicitly), no fast-math, OpenMP over the outermost lattice axis (each
node's arithmetic is independent of the thread count).
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
LIBS = {"f64": "liboracle_f64.so", "f32": "liboracle_f32.so", "plain": "liboracle_plain.so"}
DEFINES = {"f64": ["-DREAL=double"], "f32": ["-DREAL=float"],
           "plain": ["-DREAL=double", "-DPLAIN"]}


def lib_path(kind: str) -> str:
    return os.path.join(HERE, LIBS[kind])


def build(force: bool = True) -> None:
    for kind in LIBS:
        out = lib_path(kind)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-ffp-contract=off", "-fno-fast-math", *DEFINES[kind],
               "-Wall", "-Wextra", "-Wno-unused-parameter",
               SRC, "-o", out + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build(force=True)
    print("built", [lib_path(k) for k in LIBS], file=sys.stderr)
