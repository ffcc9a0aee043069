"""Compile the oracle's C part (oracle/direct.c -> oracle/_direct.so) with gcc.

Test infrastructure only: the library never loads it.

    python -m oracle.build
"""
from __future__ import annotations

import shutil
import subprocess
from pathlib import Path

HERE = Path(__file__).resolve().parent
SRC = HERE / "direct.c"
OUT = HERE / "_direct.so"


def build(verbose: bool = True) -> Path:
    cc = shutil.which("gcc") or "gcc"
    tmp = OUT.with_suffix(".so.tmp")
    cmd = [cc, "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
           str(SRC), "-o", str(tmp), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"gcc failed for {SRC.name}:\n{r.stdout}\n{r.stderr}")
    tmp.replace(OUT)
    if verbose:
        print(f"built {OUT}")
    return OUT


if __name__ == "__main__":
    build()
