"""Compile the FP64 oracle into ``oracle/liboracle.so`` (test infrastructure).

Plain gcc, C11, OpenMP over rows, no fast-math and no floating-point
contraction, so that every double operation is the one written in the source.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, out: str = OUT, sanitize: bool = False) -> str:
    """Compile the oracle into `out`.  sanitize=True builds it with
    AddressSanitizer and UndefinedBehaviorSanitizer (any report aborts); the
    process that loads such a build must preload libasan and libubsan."""
    cmd = [
        "gcc", "-O1" if sanitize else "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
        "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wno-unused-variable",
        *(SANITIZE if sanitize else []),
        SRC, "-o", out + ".tmp", "-lm",
    ]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
