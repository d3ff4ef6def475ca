"""Build ``tests/native/server_stress``: the serving-loop stress check.

The library's sources and the stress program are compiled with a sanitizer on their
host code only (``-Xarch_host`` before the sanitizer flag; the gfx950 device
code is built as for the library), and linked with the C oracle (built
without OpenMP, so its loops run on the calling thread).  Objects go to
``_build/asan``.  ``python tests/native/build_stress.py`` builds it;
``tests/test_gpu_server_stress.py`` runs it.

AddressSanitizer is the one used.  Built with ThreadSanitizer instead
(``build("thread")``), the process finds no GPU: the HIP runtime's
hipGetDeviceCount returns hipErrorNoDevice before any of this code runs.
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
from paper_2510_03631_amd import build as lib  # noqa: E402

SANITIZERS = {"thread": "tsan", "address": "asan"}


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"failed: {' '.join(cmd)}\n{res.stdout}{res.stderr}")


def build(sanitizer: str = "address") -> str:
    tag = SANITIZERS[sanitizer]
    OUT = os.path.join(HERE, "server_stress")
    OBJ = os.path.join(ROOT, "_build", tag)
    SAN_HOST = ["-Xarch_host", f"-fsanitize={sanitizer}"]
    if sanitizer == "address":
        SAN_HOST += ["-Xarch_host", "-fno-omit-frame-pointer"]
    os.makedirs(OBJ, exist_ok=True)
    flags = [f for f in lib.COMMON if f != "-O3"] + ["-O1", "-g"] + SAN_HOST
    srcs = sorted(glob.glob(os.path.join(lib.CSRC, "*.hip")))
    jobs = []
    for src in srcs:
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append(([lib.hipcc()] + flags + ["-c", src, "-o", obj], obj))
    drv = os.path.join(OBJ, "server_stress.o")
    jobs.append(([lib.hipcc(), "-O1", "-g", "-std=c++17", "-I", lib.INCLUDE, "-D__HIP_PLATFORM_AMD__",
                  "-pthread"] + SAN_HOST + ["-c", os.path.join(HERE, "server_stress.cpp"), "-o", drv],
                 drv))
    with cf.ThreadPoolExecutor(max_workers=8) as ex:
        list(ex.map(lambda j: _run(j[0]), jobs))
    orc = os.path.join(OBJ, "pir_oracle.o")
    _run(["gcc", "-O1", "-g", "-std=c11", f"-fsanitize={sanitizer}", "-c",
          os.path.join(ROOT, "oracle", "pir_oracle.c"), "-o", orc])
    _run([lib.hipcc(), f"--offload-arch={lib.ARCH}", "-pthread"] + SAN_HOST +
         ["-o", OUT] + [o for _, o in jobs] + [orc])
    return OUT


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else "address"))
