"""The library's HIP kernels, compiled for the host against an emulation of
the HIP subset they use (tests/cpu_hip) with AddressSanitizer, driven through
the C ABI on small seeded cases: every device-memory access is checked
against its allocation, every allocation starts filled with garbage bytes
(so a read before write of an index faults and of a value breaks parity),
and the results must match the oracle (neighbours and CSR structure
bit-exact, values and solves to the GPU-test tolerances).

The default run checks one 3-D case with ghosts; RT_CPU_FULL=1 runs every
workload family and all precision/preconditioner combinations."""
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ASAN = "/usr/lib/gcc/x86_64-linux-gnu/11/libasan.so"


@pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(ASAN),
                    reason="needs g++ and libasan")
def test_kernels_under_asan_match_oracle():
    sys.path.insert(0, os.path.join(HERE, "cpu_hip"))
    import build_cpu
    lib = build_cpu.build()
    env = dict(os.environ)
    env.update(RT_CPU_LIB=lib, LD_PRELOAD=ASAN,
               ASAN_OPTIONS="detect_leaks=0:max_malloc_fill_size=2147483647:malloc_fill_byte=190")
    if os.environ.get("RT_CPU_FULL") != "1":
        env.update(RT_CPU_QUICK="1", RT_CPU_CASES="marshak3d_8")
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "cpu_hip", "run_cases.py")],
                       env=env, capture_output=True, text=True, timeout=1800)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-6000:]
    assert "all cases ok" in r.stdout
