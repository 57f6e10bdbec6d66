"""AddressSanitizer + UndefinedBehaviorSanitizer run of the host code.

The oracle (oracle/oracle.c) and the library's host code (sector builder,
C ABI, runtime: every .cpp under csrc/) are rebuilt with both sanitizers
(host code only; the kernels and their launch stubs are the normal build's
objects) and the CPU tests of the oracle pins and the sector builder run
against those builds in a child process with the sanitizer runtime
preloaded.  Any sanitizer report fails the test.  CPU only.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2605_07621_amd")
LLVM = "/opt/rocm/llvm"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
# tests of the oracle and of the host sector builder, without the two
# headline-size cases (165M and 155M positions, too slow under the sanitizers)
SUBSET = ["tests/test_oracle_pins.py", "tests/test_sector_builder.py", "-k",
          "not hubbard16 and not chain_16 and not j1j2_6x5 and not workload_block and not whole_row "
          "and not spin_tile_tuning_host and not heisenberg16_dense"]


def _asan_runtime():
    found = sorted(glob.glob(os.path.join(LLVM, "lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")))
    return found[-1] if found else None


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"


def _build_oracle(out):
    _run([os.path.join(LLVM, "bin/clang"), "-O1", "-g", "-std=c99", "-fopenmp", "-fPIC", "-shared",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
          "-DORC_PLANT=0", "-o", out, os.path.join(ROOT, "oracle", "oracle.c"), "-lm",
          "-L" + os.path.join(LLVM, "lib"), "-Wl,-rpath," + os.path.join(LLVM, "lib")])


def _build_library(tmp, out):
    import concurrent.futures as cf
    sys.path.insert(0, PKG)
    import build as pkg_build   # the package's own source list
    sys.path.pop(0)
    hosts = [s for s in pkg_build.SOURCES if s.endswith(".cpp")]
    devs = [os.path.join(pkg_build.BUILD, os.path.splitext(s)[0] + ".o") for s in pkg_build.SOURCES
            if s.endswith(".hip")]
    if not all(os.path.exists(d) for d in devs):
        pkg_build.build()

    def comp(src):
        obj = os.path.join(tmp, os.path.splitext(src)[0] + ".o")
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950"] + SAN_HOST +
             ["-c", os.path.join(pkg_build.CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(comp, hosts))
    _run([os.path.join(LLVM, "bin/clang++"), "-shared", "-fPIC", "-o", out] + objs + devs +
         ["-fsanitize=address,undefined", "-shared-libsan", "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
          "-lamdhip64", "-lrocsolver", "-lrocblas", "-lpthread"])


def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    rt = _asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("no clang sanitizer runtime or hipcc in this image")
    orc = str(tmp_path / "liboracle_san.so")
    lib = str(tmp_path / "libecut_san.so")
    _build_oracle(orc)
    _build_library(str(tmp_path), lib)
    env = dict(os.environ)
    env.update(LD_PRELOAD=rt, ORACLE_LIB=orc, ECUT_LIB=lib, OMP_NUM_THREADS="4",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"] +
                       SUBSET, cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-6000:]
    assert "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in r.stdout
