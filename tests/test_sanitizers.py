"""Sanitizer runs of the oracle on the CPU (no GPU).

  * the oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
    (gcc, halting on the first report) runs the oracle pins in a child
    process (every tests/test_oracle_*.py that is neither GPU nor slow);
  * ThreadSanitizer (LLVM clang with its OpenMP runtime and the Archer tool,
    which teaches it OpenMP's synchronisation) over the oracle's OpenMP loops:
    the flux, vector flux, bands, walk variant, particle trace, background
    shell and adjoint, on four threads, binary64 and mirror mode
    (tests/oracle_tsan_driver.c); and, so that a clean report means
    something, the same setup flags a planted race.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests")
CLANG = "/opt/rocm/llvm/bin/clang"
LLVM_LIB = "/opt/rocm/llvm/lib"
ARCHER = os.path.join(LLVM_LIB, "libarcher.so")


def _gcc_file(name):
    return subprocess.check_output(["gcc", "-print-file-name=" + name]).decode().strip()


@pytest.mark.slow
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    from oracle import oracle as O
    lib = O.build_library(path=str(tmp_path / "liboracle_san.so"),
                          extra=("-O1", "-g", "-fno-omit-frame-pointer",
                                 "-fsanitize=address,undefined",
                                 "-fno-sanitize-recover=undefined"))
    asan = _gcc_file("libasan.so")
    assert os.path.exists(asan)
    env = dict(os.environ, LD_PRELOAD=asan, TREVR_ORACLE_LIB=lib, PYTHONMALLOC="malloc",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    files = sorted(glob.glob(os.path.join(HERE, "test_oracle_*.py")))
    assert len(files) >= 8
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow"] + files, cwd=ROOT, env=env,
                       capture_output=True, text=True, timeout=1200)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, out
    assert " passed" in r.stdout


def _tsan_env():
    return dict(os.environ, OMP_TOOL_LIBRARIES=ARCHER, LD_LIBRARY_PATH=LLVM_LIB,
                TSAN_OPTIONS="halt_on_error=1:exitcode=66:ignore_noninstrumented_modules=1",
                OMP_NUM_THREADS="4",
                ARCHER_OPTIONS="verbose=0")


def _tsan_build(srcs, exe):
    subprocess.check_call([CLANG, "-O1", "-g", "-fopenmp", "-fsanitize=thread", "-ffp-contract=off",
                           "-D_GNU_SOURCE"] + srcs + ["-o", exe, "-lm", "-L", LLVM_LIB,
                                                      "-Wl,-rpath," + LLVM_LIB])


needs_llvm = pytest.mark.skipif(not (os.path.exists(CLANG) and os.path.exists(ARCHER)),
                                reason="LLVM clang with OpenMP and Archer not installed")


@pytest.mark.slow
@needs_llvm
def test_tsan_flags_a_planted_race(tmp_path):
    src = tmp_path / "race.c"
    src.write_text("""
#include <stdio.h>
int main(void) {
  double sum = 0.0;
#pragma omp parallel for
  for (int i = 0; i < 100000; ++i) sum += i; /* no reduction: a data race */
  printf("%g\\n", sum);
  return 0;
}
""")
    exe = str(tmp_path / "race")
    _tsan_build([str(src)], exe)
    r = subprocess.run([exe], env=_tsan_env(), capture_output=True, text=True, timeout=120)
    assert r.returncode == 66 and "data race" in r.stderr, r.stderr[-2000:]


@pytest.mark.slow
@needs_llvm
def test_oracle_openmp_loops_under_tsan(tmp_path):
    exe = str(tmp_path / "oracle_tsan")
    _tsan_build([os.path.join(ROOT, "oracle", "trevr_oracle.c"),
                 os.path.join(HERE, "oracle_tsan_driver.c")], exe)
    r = subprocess.run([exe, "1200", "4"], env=_tsan_env(), capture_output=True, text=True,
                       timeout=900)
    assert r.returncode == 0, (r.returncode, r.stdout[-1000:], r.stderr[-4000:])
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert "driver done: ok" in r.stdout
