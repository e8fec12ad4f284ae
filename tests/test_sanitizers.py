"""The oracle and libmsp's host code under AddressSanitizer and UndefinedBehavior-
Sanitizer (CPU only). The oracle runs its pin tests instrumented; libmsp's C ABI runs
every check that needs no device, with handles that point at freed and at foreign
memory and with double frees: the library must reject them without reading through
them (a registry of live handles), and no sanitizer may report anything."""
import os
import shutil

import pytest

import sanitizers as san

REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _clean(out):
    return not any(r in out for r in REPORTS)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = san.build_oracle(str(tmp_path / "libmsp_oracle_asan.so"))
    preload = san.gcc_runtime("libasan.so") + ":" + san.gcc_runtime("libubsan.so")
    tests = ["tests/test_oracle_pins.py", "tests/test_oracle_plasticity.py",
             "tests/test_oracle_activity.py", "tests/test_plasticity_cpu.py"]
    rc, out = san.run_child(["-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                             "-m", "not gpu", *tests], preload,
                            extra_env={"MSP_ORACLE_LIB": lib, "OMP_NUM_THREADS": "4"})
    tail = out[-3000:]
    assert rc == 0, tail
    assert _clean(out), tail
    assert " passed" in out, tail


@pytest.mark.skipif(san.clang_asan_runtime() is None or
                    not os.path.exists(san.build_lib.HIPCC), reason="no hipcc / ASan runtime")
def test_libmsp_host_code_under_asan_ubsan(tmp_path):
    lib = san.build_libmsp(str(tmp_path / "libmsp_asan.so"))
    rc, out = san.run_child([os.path.join(san.ROOT, "tests", "abi_sanitized_child.py"), lib],
                            san.clang_asan_runtime())
    tail = out[-3000:]
    assert rc == 0, tail
    assert _clean(out), tail
    assert "abi checks under sanitizers: ok" in out, tail
