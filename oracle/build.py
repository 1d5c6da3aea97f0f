"""Build the C oracle into oracle/libising_oracle.so (test infrastructure).

The oracle is plain C compiled with gcc. Floating-point contraction is off so
that the threshold table is evaluated exactly in the written order.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ising_oracle.c")
LIB = os.path.join(HERE, "libising_oracle.so")


def compile_oracle(src=SRC, out=LIB, extra_flags=()):
    """Compile `src` into the shared library `out`; returns `out`."""
    cmd = ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
           "-ffp-contract=off", "-fno-fast-math", *extra_flags, "-o", out, src, "-lm"]
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    print(compile_oracle(), file=sys.stderr)
