"""Build the in-tree shared library ``libhs.so`` for gfx950.

HIP sources (``csrc/*.hip``) are compiled with hipcc for gfx950; the host
runtime (``csrc/*.cpp``) with g++ (it needs libquadmath for correctly rounded
twiddles and Gaussian tables, and -ffp-contract=off so the encoding's
floating-point operations are exactly the specified ones).  Everything is
linked by hipcc into one shared object next to this file.
"""
import concurrent.futures
import glob
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libhs.so")
OBJ = os.path.join(HERE, "_build")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HIPCC_FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-ffp-contract=off"]
GXX_FLAGS = ["-O2", "-std=gnu++17", "-fPIC", "-ffp-contract=off", "-Wall", "-Wno-unused-function", "-Wno-unused-result",
             "-D__HIP_PLATFORM_AMD__", "-I" + os.path.join(ROCM, "include")]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l and l.strip())
    if p.returncode != 0:
        raise RuntimeError("command failed: %s\n%s" % (" ".join(cmd), out))
    return out


def build(verbose=False):
    os.makedirs(OBJ, exist_ok=True)
    jobs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append(["hipcc"] + HIPCC_FLAGS + ["-c", src, "-o", obj])
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(OBJ, os.path.basename(src) + ".o")
        jobs.append(["g++"] + GXX_FLAGS + ["-c", src, "-o", obj])
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out:
                print(out)
    objs = [j[-1] for j in jobs]
    tmp = OUT + ".tmp%d" % os.getpid()
    _run(["hipcc", "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs +
         ["-lquadmath", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64"])
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
