"""Compile the FP64 C oracle into ``oracle/liboracle_eed4.so`` (test infrastructure)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "eed4_oracle.c")
LIB = os.path.join(HERE, "liboracle_eed4.so")


def build_sanitized(out: str, verbose: bool = False) -> str:
    """The same oracle with AddressSanitizer and UndefinedBehaviorSanitizer (host code,
    gcc), aborting on the first finding; for running the pins under the sanitizers.
    The library must be loaded into a process that has libasan preloaded."""
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-Wall", "-Wextra", "-fopenmp", "-shared", "-fPIC",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-o", out, SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    return out


def build(verbose: bool = False) -> str:
    cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fopenmp", "-shared",
           "-fPIC", "-o", LIB + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
