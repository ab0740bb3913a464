"""Build oracle/liboracle.so from oracle/oracle.c with gcc (FP64, OpenMP, no fast-math).

Test infrastructure only: the oracle verifies the product path and is never part of it.
"""
from __future__ import annotations

import subprocess
import sys
from pathlib import Path

HERE = Path(__file__).resolve().parent


def build(verbose: bool = False, out: Path | None = None, native: bool = False) -> Path:
    """Compile oracle.c.  native=True adds -O3 -march=native for timing runs on the
    machine that compiles it (the CPU-baseline leg builds such a copy in a
    temporary directory on the host it times); the shipped test library is -O2
    for any x86-64 host."""
    src = HERE / "oracle.c"
    out = Path(out) if out is not None else HERE / "liboracle.so"
    tmp = out.with_name(out.name + ".tmp")
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", *opt, "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-Wall", "-Wextra", "-o", str(tmp), str(src), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
