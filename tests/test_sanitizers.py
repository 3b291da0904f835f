"""AddressSanitizer + UndefinedBehaviorSanitizer builds of host code, run on the CPU:

* the FP64 oracle (g++ -fsanitize=address,undefined), under its pin tests;
* the library's host code (the C ABI's argument checks, topology and workspace carving, the Umeyama solve,
  the tracker's scratch sizing, the block-sparse and tile-sparse solvers' symbolic analyses): every source compiled by
  hipcc with the sanitizers on the host side only (-Xarch_host before each -fsanitize=), under the
  host-only ABI and analysis tests.

Each run is a child pytest process with the sanitizer runtime preloaded and the instrumented library named
by DS3_ORACLE_LIB / DS3_LIB; any sanitizer report fails the test. No GPU is used."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _child_pytest(env, files, timeout=900):
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *files]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, out
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer"):
        assert marker not in r.stderr, out
    return r


@pytest.mark.slow
def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_san.so")
    subprocess.check_call(["g++", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp", "-shared", "-fPIC",
                           "-std=c++17", os.path.join(ROOT, "oracle", "ds3_oracle.cpp"), "-o", lib])
    asan = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    env = dict(os.environ, DS3_ORACLE_LIB=lib, LD_PRELOAD=asan,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _child_pytest(env, ["tests/test_oracle_sim3.py", "tests/test_oracle_gn.py", "tests/test_oracle_match.py",
                        "tests/test_oracle_calib.py", "tests/test_oracle_track.py", "tests/test_oracle_gauge.py"])


@pytest.mark.slow
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    from paper_2605_30488_amd import _build
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined", "-Xarch_host",
           "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(src)[0] + ".o"))
        cmd = [_build.HIPCC, *_build.FLAGS, *_build.EXTRA.get(src, []), *san, "-x", "hip", "-c",
               os.path.join(_build.CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(min(8, os.cpu_count() or 4)) as ex:
        objs = list(ex.map(compile_one, _build.SOURCES))
    lib = str(tmp_path / "libds3_san.so")
    r = subprocess.run([_build.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *san, "-shared-libsan", *objs,
                        "-o", lib], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    rt = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rt:
        pytest.skip("clang's AddressSanitizer runtime is not installed")
    env = dict(os.environ, DS3_LIB=lib, LD_PRELOAD=rt[0],
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    _child_pytest(env, ["tests/test_abi.py", "tests/test_spchol_host.py", "tests/test_tilechol_host.py"])
