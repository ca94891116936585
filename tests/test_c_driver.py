"""The C ABI from a plain C program (tests/c_driver/gbr_c_driver.c: only
include/gbr.h and the HIP runtime API; no Python binding, no torch).

Host-only here: the driver is built (build() builds it; this test builds it
when missing), and it rejects bad usage and unreadable input before any HIP
call.  The GPU run against the oracle is in test_c_driver_gpu.py.
"""
import os
import struct
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EXE = os.path.join(ROOT, "tests", "c_driver", "gbr_c_driver")


@pytest.fixture(scope="module")
def driver():
    if not os.path.exists(EXE):
        import importlib.util
        spec = importlib.util.spec_from_file_location(
            "gbr_c_driver_build", os.path.join(ROOT, "tests", "c_driver", "build.py"))
        m = importlib.util.module_from_spec(spec)
        spec.loader.exec_module(m)
        m.build()
    return EXE


def test_usage_and_bad_input(driver, tmp_path):
    r = subprocess.run([driver], capture_output=True, text=True, timeout=60)
    assert r.returncode == 2 and "usage" in r.stderr
    r = subprocess.run([driver, str(tmp_path / "missing.bin"), str(tmp_path / "o.bin")],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    bad = tmp_path / "short.bin"
    bad.write_bytes(struct.pack("<4i", 8, 8, 0, 0))          # header cut short
    r = subprocess.run([driver, str(bad), str(tmp_path / "o.bin")], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2 and "short header" in r.stderr
    huge = tmp_path / "huge.bin"
    huge.write_bytes(struct.pack("<4i8d", 1 << 14, 1 << 14, 0, 0, 0, 1, 0, 1, 1.4, 0, 0.72, 0.2))
    r = subprocess.run([driver, str(huge), str(tmp_path / "o.bin")], capture_output=True,
                       text=True, timeout=60)
    assert r.returncode == 2 and "bad grid" in r.stderr
