"""Build librdpdhg.so for gfx950 from the HIP sources in csrc/ (in-tree).

The FFT-carrying kernels are instantiated once per grid size: kernels_inst.hip
is compiled nine times with -DRD_LOGN=4..12 (N = 16..4096), in parallel.
Usage: python -m paper_2305_03945_amd.build [-j JOBS]
"""
import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "librdpdhg.so")
ARCH = "gfx950"
LOGNS = range(4, 13)

HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# Packed FP32 instructions are disabled for all device code.
DEVICE_FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I" + CSRC, "-I" + os.path.join(ROOT, "include")]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines()
                    if "unknown target feature" not in l and "packed-fp32-ops" not in l
                    and "warning generated" not in l and l.strip())
    if p.returncode != 0:
        raise RuntimeError("build step failed: %s\n%s" % (" ".join(cmd), out))
    return out


def jobs_list():
    jobs = []
    for l in LOGNS:
        jobs.append((os.path.join(CSRC, "kernels_inst.hip"), os.path.join(BUILD, "kernels_%d.o" % l),
                     ["-DRD_LOGN=%d" % l]))
    jobs.append((os.path.join(CSRC, "kernels_misc.hip"), os.path.join(BUILD, "kernels_misc.o"), []))
    jobs.append((os.path.join(CSRC, "runtime.cpp"), os.path.join(BUILD, "runtime.o"), []))
    return jobs


def build(jobs=None, verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(16, os.cpu_count() or 4)
    work = jobs_list()

    def compile_one(item):
        src, obj, extra = item
        cmd = [HIPCC] + DEVICE_FLAGS + extra + ["-c", src, "-o", obj]
        return _run(cmd)

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        for out in ex.map(compile_one, work):
            if verbose and out:
                print(out)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + [o for _, o, _ in work])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.j, a.v))
    sys.exit(0)
