"""Build the FP64 CPU oracle shared library (test infrastructure only).

``python -m oracle.build`` or ``oracle.build.build()`` compiles
``lb_oracle.c`` with gcc into ``liblb_oracle.so`` beside it.  The flags keep
every floating-point operation rounding as written (no FMA contraction, no
fast-math); OpenMP only splits the per-site loops across threads.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liblb_oracle.so")
SRC = os.path.join(HERE, "lb_oracle.c")


def build(verbose: bool = False) -> str:
    cmd = [
        "gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
        "-fPIC", "-shared", "-Wall", "-Wextra", "-o", LIB + ".tmp", SRC, "-lm",
    ]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def ensure_built() -> str:
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        build()
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
