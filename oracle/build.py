"""Build the C oracle (test infrastructure) into ``oracle/_build/``.

gcc -O3 -march=native -fopenmp -ffp-contract=off, no fast-math: IEEE double with
round-to-nearest and no contraction of a*b+c into a fused multiply-add.
"""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD = os.path.join(HERE, "_build")

LIBS = {
    "libsw2d_oracle.so": ["sw2d_oracle.c"],
    "libsor_oracle.so": ["sor_oracle.c"],
}

CFLAGS = ["-O3", "-march=native", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
          "-std=c11", "-fPIC", "-shared", "-Wall", "-Wextra"]


def lib_path(name: str) -> str:
    return os.path.join(BUILD, name)


def build(force: bool = True, verbose: bool = False) -> None:
    os.makedirs(BUILD, exist_ok=True)
    for lib, srcs in LIBS.items():
        out = lib_path(lib)
        paths = [os.path.join(HERE, s) for s in srcs]
        if not force and os.path.exists(out) and all(
                os.path.getmtime(out) >= os.path.getmtime(p) for p in paths):
            continue
        tmp = out + f".tmp{os.getpid()}"
        cmd = ["gcc", *CFLAGS, *paths, "-o", tmp, "-lm"]
        if verbose:
            print(" ".join(cmd), file=sys.stderr)
        subprocess.run(cmd, check=True)
        os.replace(tmp, out)


if __name__ == "__main__":
    build(force=True, verbose=True)
