"""Build oracle/liboracle.so from oracle/oracle.c with gcc (FP64, OpenMP, no fast-math).

Test infrastructure only: the oracle verifies the product path and is never part of it.
"""
from __future__ import annotations

import os
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


def build_sanitized(verbose: bool = False, out: Path | None = None) -> Path:
    """oracle/liboracle_san.so: oracle.c under ASan + UBSan, built with the ROCm
    clang so that one shared sanitizer runtime serves it and the sanitized host
    library of the product (paper_2104_03293_amd/build.py, build_sanitized) in
    the same Python process."""
    src = HERE / "oracle.c"
    out = Path(out) if out is not None else HERE / "liboracle_san.so"
    tmp = out.with_name(out.name + ".tmp")
    llvm = Path(os.environ.get("SV_CLANG_DIR", "/opt/rocm/llvm/bin"))
    cmd = [str(llvm / "clang"), "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
           "-shared-libsan", "-Wall", "-Wextra", "-o", str(tmp), str(src), "-lm",
           f"-L{llvm.parent / 'lib'}", f"-Wl,-rpath,{llvm.parent / 'lib'}"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
