"""Build the HIP library ``libvmcpeps.so`` for gfx950 in-tree.

    python -m paper_1908_09359_amd.build

Every HIP translation unit is compiled with packed-FP32 instruction selection
disabled (see the design notes); objects are linked into one shared library
next to this file.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "libvmcpeps.so")
BUILD = os.path.join(ROOT, "_build")

# (source, object name, extra flags): the phase kernels compile once per working type
SOURCES = [("vp_kernels.hip", "vp_kernels_f64", ["-DVP_KERNEL_UNIT=0"]),
           ("vp_kernels.hip", "vp_kernels_f32", ["-DVP_KERNEL_UNIT=1"]),
           ("vp_sr.hip", "vp_sr", []), ("vp_net.hip", "vp_net", []), ("vp_sis.hip", "vp_sis", []), ("vp_su.hip", "vp_su", []), ("vp_cols.hip", "vp_cols", []),
           ("vp_api.cpp", "vp_api", [])]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("VP_OFFLOAD_ARCH", "gfx950")

FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
    "-I", os.path.join(ROOT, "include"),
]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd))
    return r


def build(verbose=False):
    os.makedirs(BUILD, exist_ok=True)
    objs, cmds = [], []
    for src, name, extra in SOURCES:
        obj = os.path.join(BUILD, name + ".o")
        cmds.append([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj] + FLAGS + extra)
        objs.append(obj)
    if verbose:
        for cmd in cmds:
            print(" ".join(cmd), flush=True)
    # the translation units are independent: compile them side by side
    with ThreadPoolExecutor(max_workers=min(len(cmds), os.cpu_count() or 1)) as pool:
        list(pool.map(_run, cmds))
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    _run(cmd)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
