"""Build libmpcd.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2212_11878_amd.csrc.build  (or import and call build()).
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
LIB_PATH = os.path.join(PKG, "libmpcd.so")
SOURCES = ["mpcd_kernels.hip", "mpcd_engine.hip", "mpcd_host.hip"]
# host code of the CPU leg: fused multiply-add and AVX2 (x86-64-v3; every
# EPYC and every Xeon since Haswell), so fmaf is one instruction
EXTRA_FLAGS = {"mpcd_host.hip": ["-Xarch_host", "-mfma", "-Xarch_host", "-mavx2"]}
HEADERS = ["mpcd_dev.h", "mpcd_launch.h"]
ARCH = os.environ.get("MPCD_OFFLOAD_ARCH", "gfx950")


def _hipcc():
    return shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


def build(verbose=False, jobs=2):
    """Compile every HIP source for gfx950 and link libmpcd.so next to the
    package.  Always recompiles."""
    bdir = os.path.join(PKG, "_build")
    os.makedirs(bdir, exist_ok=True)
    flags = ["-O3", "--offload-arch=" + ARCH, "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", HERE, "-Wall"]
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(bdir, src.replace(".hip", ".o"))
        cmd = [_hipcc()] + flags + EXTRA_FLAGS.get(src, []) + ["-c", os.path.join(HERE, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    for p in procs:
        _wait(p, verbose)
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = [_hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def _wait(item, verbose):
    src, p = item
    out, _ = p.communicate()
    text = "\n".join(l for l in out.decode(errors="replace").splitlines()
                     if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError("hipcc failed on %s:\n%s" % (src, text))
    if verbose and text.strip():
        print(text)


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
