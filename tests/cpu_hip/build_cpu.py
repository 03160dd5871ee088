"""Build the library's HIP sources for the CPU (tests/cpu_hip shim headers in
place of the HIP runtime and hipcub) with AddressSanitizer, so kernel
indexing can be checked against real allocation bounds on the host.

Test infrastructure: the product library is built by paper_2001_11606_amd/build.py.
"""
import os
import sys
import subprocess
import concurrent.futures as cf

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2001_11606_amd", "csrc")
OUT_DIR = os.environ.get("RT_CPU_BUILD_DIR") or os.path.join(ROOT, "_build", "cpu_hip")
LIB = os.path.join(OUT_DIR, "librt_cpu.so")
sys.path.insert(0, ROOT)
from paper_2001_11606_amd.build import SOURCES  # noqa: E402  (the same source list as the HIP build)
FLAGS = ["-x", "c++", "-std=c++20", "-O1", "-g", "-fPIC", "-fno-omit-frame-pointer",
         "-fsanitize=address", "-ffp-contract=off", "-pthread", "-w",
         # always take the two-level reduction path, which large GPU runs use
         "-DRT_PARTIAL_FOLD_MIN=4", "-DRT_POOL_POISON",
         "-I" + HERE, "-I" + os.path.join(ROOT, "include")]


def _one(src):
    obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
    r = subprocess.run(["g++"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(f"g++ failed on {src}:\n{r.stderr[-4000:]}")
    return obj


def build():
    os.makedirs(OUT_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(6) as ex:
        objs = list(ex.map(_one, SOURCES))
    r = subprocess.run(["g++", "-shared", "-o", LIB, "-x", "none"] + objs
                       + ["-fsanitize=address", "-pthread"],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr[-4000:])
    return LIB


if __name__ == "__main__":
    print(build())
