"""Compile the FP64 CPU oracle (test infrastructure only).

Two shared libraries come from the one source file:
  liboracle.so     -- `real` = double
  liboracle_cs.so  -- `real` = double _Complex (complex-step derivatives)
No fused multiply-add contraction (-ffp-contract=off), so the indicator test
is evaluated exactly as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lbm_oracle.c")
FLAGS = ["-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared"]


def lib_path(complex_step=False):
    return os.path.join(HERE, "liboracle_cs.so" if complex_step else "liboracle.so")


def build(force=True):
    for cs in (False, True):
        out = lib_path(cs)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(SRC):
            continue
        cmd = ["gcc", *FLAGS, *(["-DORACLE_COMPLEX"] if cs else []), SRC, "-o", out + ".tmp", "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(out + ".tmp", out)


if __name__ == "__main__":
    build()
    print("built", lib_path(False), lib_path(True))
