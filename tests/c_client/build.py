"""Compile the plain C client of the library (gcc, C99) into tests/c_client/_build/."""

from __future__ import annotations

import os
import shutil
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "sw2d_client.c")
BIN = os.path.join(HERE, "_build", "sw2d_client")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build() -> str:
    os.makedirs(os.path.dirname(BIN), exist_ok=True)
    cc = shutil.which("gcc") or "gcc"
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROCM, "include"), SRC,
           "-L", os.path.join(ROOT, "paper_1711_04471_amd"), "-lsw2d",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64",
           # the library is found next to the package wherever the tree is copied
           "-Wl,-rpath,$ORIGIN/../../../paper_1711_04471_amd", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-o", BIN]
    subprocess.run(cmd, check=True)
    return BIN


if __name__ == "__main__":
    print(build())
