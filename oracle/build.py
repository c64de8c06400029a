"""Compile the CPU oracle (plain C, gcc) into oracle/_build/liboracle.so.

No fused multiply-add and no fast-math, so every operation rounds once to
nearest-even and results are reproducible across machines.
"""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def lib_path() -> str:
    return os.path.join(HERE, "_build", "liboracle.so")


def build(verbose: bool = False, mutant: int = 0, out: str | None = None) -> str:
    """Compile the oracle.  mutant=k > 0 builds the k-th planted-mistake
    variant (test-suite only) into `out`."""
    out = out or lib_path()
    os.makedirs(os.path.dirname(out), exist_ok=True)
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-fno-fast-math",
           "-Wall", "-Wno-unused-function", "-pthread", "-DORA_MUTANT=%d" % int(mutant),
           os.path.join(HERE, "ata_oracle.c"), "-lm", "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
