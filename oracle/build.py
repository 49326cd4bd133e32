"""Build the C oracle (test infrastructure) into oracle/liboracle.so with gcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lb_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
CHECK_SRC = os.path.join(HERE, "sanitize_check.c")
CHECK_EXE = os.path.join(HERE, "sanitize_check")


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra",
           "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


def build_sanitize_check(verbose: bool = False) -> str:
    """The oracle and a program calling all its entry points, built with
    AddressSanitizer and UndefinedBehaviorSanitizer (host code only; any
    report aborts the run with a nonzero exit)."""
    cmd = ["gcc", "-O1", "-g", "-fopenmp", "-std=c11", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-o", CHECK_EXE, CHECK_SRC, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return CHECK_EXE


if __name__ == "__main__":
    print(build(verbose=True))
