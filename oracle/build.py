"""Compile the C half of the oracle (test infrastructure) into librga_oracle.so."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rga_oracle.c")
LIB = os.path.join(HERE, "librga_oracle.so")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wno-misleading-indentation", SRC, "-o", LIB, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return LIB


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The same source with AddressSanitizer and UndefinedBehaviorSanitizer
    (host code only; no OpenMP, so the sanitizers see one thread), for the
    CPU tests that run the oracle under them."""
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           "-fno-omit-frame-pointer", "-fPIC", "-shared", "-Wall", "-Wno-misleading-indentation",
           "-Wno-unknown-pragmas", SRC, "-o", out, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
