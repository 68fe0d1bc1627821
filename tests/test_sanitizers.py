"""AddressSanitizer + UndefinedBehaviorSanitizer runs on the CPU (no GPU needed).

* The oracle (oracle/oracle.c) is compiled with gcc and the sanitizers into a driver that calls
  every one of its functions on small inputs (tests/sanitize/oracle_driver.c).
* The library's host code is compiled with the sanitizers on its host side only (the device code
  is built as usual, without them) and linked into a driver that runs the host-side logic of the
  C ABI: argument validation of every entry point, GLL tables, the tuning table, the CSR inverse of
  a numbering, workspace sizing (tests/sanitize/abi_driver.cpp).  That build compiles every source
  again, so this test takes about a minute.

Both drivers exit non-zero on a failed check; a sanitizer report aborts the run (no recovery) and
leak detection is on."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2504_07042_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe, marker):
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=ENV)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert marker in r.stdout
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr


def test_oracle_under_sanitizers():
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "oracle_driver")
        subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-Wall", "-Wno-unknown-pragmas", "-o", exe,
                        os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_driver.c"), "-lm"],
                       check=True)
        _run(exe, "oracle-sanitize: ok")


def test_abi_host_code_under_sanitizers():
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm compilers not found")
    from paper_2504_07042_amd import build as hipbuild
    # the sanitizers apply to the host pass only (each -fsanitize= behind -Xarch_host)
    host_san = ["-Xarch_host", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    flags = ["-O1", "-std=c++17", "-fPIC", f"--offload-arch={hipbuild.ARCH}", "-Xclang", "-target-feature",
             "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include")] + host_san
    with tempfile.TemporaryDirectory() as td:
        def compile_one(src):
            obj = os.path.join(td, src + ".o")
            lang = ["-x", "hip"] if src.endswith(".cpp") else []
            r = subprocess.run([HIPCC] + flags + lang + ["-c", os.path.join(CSRC, src), "-o", obj],
                               capture_output=True, text=True)
            assert r.returncode == 0, r.stderr[-3000:]
            return obj
        srcs = sorted(hipbuild.SOURCES, key=lambda s: s not in hipbuild.LDS_SOURCES)
        with cf.ThreadPoolExecutor(max_workers=min(len(srcs), os.cpu_count() or 2)) as ex:
            objs = list(ex.map(compile_one, srcs))
        drv = os.path.join(td, "abi_driver.o")
        subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                        "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-c",
                        os.path.join(HERE, "abi_driver.cpp"), "-o", drv], check=True)
        exe = os.path.join(td, "abi_driver")
        subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", exe, drv] + objs +
                       ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"], check=True)
        _run(exe, "abi-sanitize: ok")
