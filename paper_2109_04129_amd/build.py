"""Build libhps.so (host C++ + HIP kernels for gfx950) in-tree.

    python -m paper_2109_04129_amd.build

Host modules are compiled with g++ (no FMA contraction, so the host
geometry arithmetic is reproducible), the device module with hipcc for
gfx950, and everything is linked by hipcc into paper_2109_04129_amd/libhps.so.
"""

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhps.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")

HOST_SRC = ["mesh.cpp", "tree.cpp", "efie.cpp", "aca.cpp", "symbolic.cpp", "batch.cpp", "tune.cpp", "api.cpp"]
DEVICE_SRC = ["device.hip"]

HOST_FLAGS = ["-O3", "-fPIC", "-std=c++17", "-ffp-contract=off", "-pthread", "-Wall",
              "-Wno-unused-function", "-I" + os.path.join(ROCM, "include"), "-D__HIP_PLATFORM_AMD__"]
DEVICE_FLAGS = ["-O3", "-fPIC", "-std=c++17", "--offload-arch=gfx950", "-ffp-contract=fast",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-Wno-unused-result"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout)
    return r.stdout


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    if os.path.exists(LIB):          # never leave a stale library behind a failed build
        os.remove(LIB)
    jobs = []
    for f in HOST_SRC:
        obj = os.path.join(OUT, f + ".o")
        jobs.append(["g++"] + HOST_FLAGS + ["-c", os.path.join(CSRC, f), "-o", obj])
    for f in DEVICE_SRC:
        obj = os.path.join(OUT, f + ".o")
        jobs.append([HIPCC] + DEVICE_FLAGS + ["-c", os.path.join(CSRC, f), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        outs = list(ex.map(_run, jobs))
    if verbose:
        for o in outs:
            if o.strip():
                print(o)
    objs = [os.path.join(OUT, f + ".o") for f in HOST_SRC + DEVICE_SRC]
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-pthread", "-ldl"])
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
