"""Build the CPU oracle (test infrastructure) into oracle/liboracle.so with gcc.

build(sanitize=True, out=...) builds an AddressSanitizer + UndefinedBehavior-
Sanitizer copy (for the sanitized run of the oracle's pin tests)."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pt_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

# No FMA contraction and no fast-math: every rounding is the one written in the
# source.  Explicit fma() calls go to glibc's correctly rounded fma.
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-fno-math-errno", "-Wall", "-Wextra"]


# Sanitized build: every undefined-behaviour report is fatal.
SANITIZE = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, sanitize: bool = False, out: str = None) -> str:
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = ["gcc", *CFLAGS, *(SANITIZE if sanitize else []), SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
