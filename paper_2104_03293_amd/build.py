"""Build libsv.so (gfx950 HIP kernels + C-ABI host code) in-tree with hipcc.

    python -m paper_2104_03293_amd.build        # or: from paper_2104_03293_amd import build; build.build()
    python -m paper_2104_03293_amd.build --sanitize   # libsv_san.so, see build_sanitized()

Flags: -O3, no fast-math (the FP64 phase angles and reductions must stay
IEEE), and packed FP32 instructions disabled for the device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor
from pathlib import Path

HERE = Path(__file__).resolve().parent
CSRC = HERE / "csrc"
ROOT = HERE.parent
ARCH = os.environ.get("SV_OFFLOAD_ARCH", "gfx950")
LIB = HERE / "libsv.so"
LIB_SAN = HERE / "libsv_san.so"
# host code of the C ABI, and the entry point that allocates nothing
HOST_SRCS = [CSRC / "sv_host_core.cpp", CSRC / "sv_plan.cpp", CSRC / "sv_api.cpp", CSRC / "sv_batch.cpp",
             CSRC / "sv_noalloc.hip"]
CLANG_DIR = Path(os.environ.get("SV_CLANG_DIR", "/opt/rocm/llvm/bin"))

DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", f"--offload-arch={ARCH}", f"-I{ROOT / 'include'}"]


# AddressSanitizer + UndefinedBehaviorSanitizer for the host pass only (each
# flag behind -Xarch_host, so the gfx950 code is built exactly as in libsv.so)
_SAN = ["address", "undefined"]
HOST_SAN_FLAGS = [f for k in _SAN for f in ("-Xarch_host", "-fsanitize=" + k)] + [
    "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def _compile(src: Path, obj: Path, verbose: bool, extra=()) -> None:
    cmd = ["hipcc", *COMMON, *DEVICE_FLAGS, *extra, "-c", str(src), "-o", str(obj)]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    noise = "is not a recognized feature for this target"
    err = "\n".join(l for l in (res.stderr or "").splitlines() if noise not in l)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{err}")
    if verbose and err.strip():
        print(err)


def build(verbose: bool = False) -> Path:
    objdir = HERE / "_build"
    objdir.mkdir(exist_ok=True)
    srcs = [CSRC / "sv_kernels.hip", *HOST_SRCS]
    objs = [objdir / (s.stem + ".o") for s in srcs]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose), zip(srcs, objs)))
    tmp = HERE / "libsv.so.tmp"
    cmd = ["hipcc", f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", str(tmp), *map(str, objs)]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(LIB)
    return LIB


def build_sanitized(verbose: bool = False, out: Path | None = None) -> Path:
    """libsv_san.so: the same library with its host code (planner, program
    builder, entry points, argument checks) under ASan + UBSan, for the CPU
    tests.  The kernels object is the one of the normal build; the library is
    linked by clang++ against the shared sanitizer runtime, which the Python
    process must preload:

        LD_PRELOAD=$(/opt/rocm/llvm/bin/clang -print-file-name=libclang_rt.asan-x86_64.so) \
        ASAN_OPTIONS=detect_leaks=0 SV_LIBRARY=paper_2104_03293_amd/libsv_san.so \
        ORACLE_LIBRARY=oracle/liboracle_san.so python -m pytest tests -m "not gpu"
    """
    objdir = HERE / "_build"
    objdir.mkdir(exist_ok=True)
    kobj = objdir / "sv_kernels.o"
    if not kobj.exists():
        _compile(CSRC / "sv_kernels.hip", kobj, verbose)
    srcs = list(HOST_SRCS)
    objs = [objdir / (s.stem + "_san.o") for s in srcs]
    with ThreadPoolExecutor(max_workers=len(srcs)) as ex:
        list(ex.map(lambda so: _compile(so[0], so[1], verbose, HOST_SAN_FLAGS), zip(srcs, objs)))
    rocm = Path(os.environ.get("ROCM_PATH", "/opt/rocm"))
    out = Path(out) if out is not None else LIB_SAN
    tmp = out.with_name(out.name + ".tmp")
    san = ",".join(_SAN)
    cmd = [str(CLANG_DIR / "clang++"), "-shared", "-fPIC", f"-fsanitize={san}", "-shared-libsan", "-o", str(tmp),
           str(kobj), *map(str, objs), f"-L{rocm / 'lib'}", "-lamdhip64", f"-Wl,-rpath,{rocm / 'lib'}"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    tmp.replace(out)
    return out


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        print(build(verbose="-v" in sys.argv))
