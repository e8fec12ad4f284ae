"""Host-code sanitizer builds for the CPU test suite (test infrastructure only).

The oracle (plain C++) and the host side of libmsp (the C ABI's argument checks,
handle registry, sizing and error paths) are compiled with AddressSanitizer and
UndefinedBehaviorSanitizer; the GPU code of libmsp is compiled as usual. The
instrumented libraries are loaded into child Python processes with the sanitizer
runtime preloaded, so that any report fails the test.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2509_26193_amd import build_lib  # noqa: E402

ORACLE_SRC = os.path.join(ROOT, "oracle", "msp_oracle.cpp")
LIBMSP_SRC = os.path.join(ROOT, "paper_2509_26193_amd", "csrc", "msp.hip")


def gcc_runtime(name: str) -> str:
    return subprocess.check_output(["gcc", f"-print-file-name={name}"], text=True).strip()


def clang_asan_runtime() -> str | None:
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build_oracle(dst: str) -> str:
    """The oracle with ASan + UBSan (g++; the same arithmetic flags as its normal build)."""
    san = ["-fsanitize=address", "-fsanitize=undefined"]
    cmd = ["g++", "-O1", "-g", "-fno-omit-frame-pointer", *san, "-fno-sanitize-recover=undefined",
           "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-shared", "-fPIC",
           ORACLE_SRC, "-o", dst]
    subprocess.check_call(cmd)
    return dst


def build_libmsp(dst: str) -> str:
    """libmsp with the host code under ASan + UBSan; device code as in the normal build."""
    host = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]
    flags = [f for f in build_lib.FLAGS if f != "-Wall"]
    cmd = [build_lib.HIPCC, *flags, *host, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.dirname(LIBMSP_SRC), LIBMSP_SRC, "-o", dst]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    return dst


def run_child(args, preload: str, extra_env=None, timeout=900):
    """Run `python args...` with the sanitizer runtime preloaded; returns
    (returncode, combined output)."""
    env = dict(os.environ)
    env.update(extra_env or {})
    env["LD_PRELOAD"] = preload
    env["PYTHONMALLOC"] = "malloc"
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    p = subprocess.run([sys.executable, *args], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=timeout)
    return p.returncode, p.stdout + p.stderr
