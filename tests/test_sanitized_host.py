"""The CPU suite under AddressSanitizer + UndefinedBehaviorSanitizer.

Builds the host code of libsv (planner, program builder, entry-point argument
checks) and the C oracle with ASan + UBSan, then runs every other CPU test in a
child process that preloads the shared sanitizer runtime and loads those two
builds.  Any sanitizer report aborts the child (UBSan does not recover), which
fails this test.  No GPU is touched: the CPU tests make no compute calls.
"""
import os
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]


@pytest.mark.skipif(os.environ.get("SV_LIBRARY", "").endswith("_san.so"), reason="already the sanitized run")
def test_cpu_suite_under_asan_ubsan(tmp_path):
    from oracle import build as obuild
    from paper_2104_03293_amd import build as pbuild

    if not (pbuild.HERE / "_build" / "sv_kernels.o").exists():
        pytest.skip("the kernels object of the normal build is missing (run the package build first)")
    clang = pbuild.CLANG_DIR / "clang"
    if not clang.exists():
        pytest.skip(f"{clang} not found")
    svlib = pbuild.build_sanitized(out=tmp_path / "libsv_san.so")
    olib = obuild.build_sanitized(out=tmp_path / "liboracle_san.so")
    rt = subprocess.run([str(clang), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                        text=True, check=True).stdout.strip()
    assert Path(rt).exists(), rt
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1", SV_LIBRARY=str(svlib), ORACLE_LIBRARY=str(olib))
    log = tmp_path / "sanitized.log"
    with open(log, "w") as f:
        res = subprocess.run([sys.executable, "-m", "pytest", str(ROOT / "tests"), "-x", "-q", "-m", "not gpu",
                              "-p", "no:cacheprovider"], cwd=ROOT, env=env, stdout=f, stderr=subprocess.STDOUT,
                             timeout=1200)
    text = log.read_text()
    assert res.returncode == 0, text[-4000:]
    assert "ERROR: AddressSanitizer" not in text and "runtime error:" not in text, text[-4000:]
