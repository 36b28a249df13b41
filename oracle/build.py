"""Builds the sequential C oracle (test infrastructure) into oracle/libcskv_oracle.so with gcc."""
from __future__ import annotations

import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build() -> str:
    src = os.path.join(_HERE, "cskv_oracle.c")
    out = os.path.join(_HERE, "libcskv_oracle.so")
    tmp = out + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
                           "-o", tmp, src])
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build())
