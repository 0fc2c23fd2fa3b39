"""Host-side sanitizer runs (CPU only): the oracle's C and the library's host
code rebuilt with AddressSanitizer and UndefinedBehaviorSanitizer, and the CPU
test files that exercise them run again against those builds in a fresh
process (the sanitizer runtime preloaded).  Device code is never
instrumented: the library's kernels are compiled as usual and only its host
half carries the checks."""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2407_20474_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def run_tests(test_file, env_extra, timeout=600):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    r = subprocess.run([sys.executable, "-m", "pytest", test_file, "-q", "-x", "-m", "not gpu",
                        "-p", "no:cacheprovider"], cwd=ROOT, env=env, timeout=timeout,
                       stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    assert r.returncode == 0, r.stdout[-4000:]
    assert "passed" in r.stdout


def gcc_runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], stdout=subprocess.PIPE,
                       text=True).stdout.strip()
    if not os.path.isabs(p) or not os.path.exists(p):
        pytest.skip(f"{name} is not installed")
    return p


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                           "-fno-omit-frame-pointer", "-o", lib,
                           os.path.join(ROOT, "oracle", "zset_oracle.c"), "-lpthread"])
    pre = gcc_runtime("libasan.so") + " " + gcc_runtime("libubsan.so")
    run_tests("tests/test_oracle.py", {"LD_PRELOAD": pre, "ZSET_ORACLE_LIB": lib})


def test_host_library_under_address_and_undefined_sanitizers(tmp_path):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    rts = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not rts:
        pytest.skip("the clang AddressSanitizer runtime is not installed")
    from paper_2407_20474_amd import build as zbuild
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f for f in zbuild.CFLAGS if f != "-O3"] + ["-O1", "-g"] + host_san

    def compile_one(src):
        obj = str(tmp_path / src.replace(".hip", ".o"))
        subprocess.check_call([HIPCC, *flags, "-c", os.path.join(CSRC, src), "-o", obj],
                              stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
        return obj

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, zbuild.SOURCES))
    lib = str(tmp_path / "libzset_asan.so")
    subprocess.check_call([HIPCC, f"--offload-arch={zbuild.ARCH}", "-shared", *host_san,
                           "-Xarch_host", "-shared-libsan", "-o", lib, *objs],
                          stdout=subprocess.DEVNULL, stderr=subprocess.DEVNULL)
    undef = subprocess.run(["nm", "-u", lib], stdout=subprocess.PIPE, text=True).stdout
    assert "__asan_report" in undef and "__ubsan_handle" in undef  # the checks are compiled in
    run_tests("tests/test_library_cpu.py", {"LD_PRELOAD": rts[0], "ZSET_LIB_PATH": lib})
