"""Compile the oracle's plain-C parts with gcc (test infrastructure)."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SOURCES = {"raycast_oracle": os.path.join(HERE, "c", "raycast_oracle.c"),
           "rbf_oracle": os.path.join(HERE, "c", "rbf_oracle.c")}


def library_path(name: str) -> str:
    return os.path.join(HERE, "c", f"lib{name}.so")


def build(force: bool = True) -> None:
    for name, src in SOURCES.items():
        out = library_path(name)
        if not force and os.path.exists(out) and os.path.getmtime(out) >= os.path.getmtime(src):
            continue
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
                               "-fno-fast-math", "-Wall", "-o", tmp, src, "-lm", "-lpthread"])
        os.replace(tmp, out)


if __name__ == "__main__":
    build()
