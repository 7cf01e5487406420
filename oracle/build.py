"""Compile the CPU oracle and the brute-force checker (test infrastructure).

Two separate shared objects are built, one per source file, so that the
checker and the oracle share no compiled code.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))

TARGETS = {
    "pt2_oracle.c": "liborc_pt2.so",
    "fci_brute.c": "liborc_fci.so",
}


def build(verbose: bool = False) -> list[str]:
    out = []
    for src, lib in TARGETS.items():
        cmd = ["gcc", "-O3", "-std=c11", "-Wall", "-Wextra", "-fPIC", "-shared",
               "-D_POSIX_C_SOURCE=200809L", "-o", os.path.join(HERE, lib),
               os.path.join(HERE, src), "-lpthread", "-lm"]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        out.append(os.path.join(HERE, lib))
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
