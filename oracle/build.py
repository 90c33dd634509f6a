"""Compile the FP64 oracle into a shared library with gcc.

Plain -O2, no fast-math and no target-specific vector flags, so the result is
the IEEE double arithmetic the source states.  Test infrastructure only.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "libmpcd_oracle.so")
SOURCES = [os.path.join(HERE, "mpcd_oracle.c")]


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-D_DEFAULT_SOURCE", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", "-Wall", "-Wextra",
           "-o", tmp] + SOURCES + ["-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def ensure_built() -> str:
    """Build if the library is missing or older than its sources."""
    if os.path.exists(LIB_PATH):
        lib_t = os.path.getmtime(LIB_PATH)
        srcs = SOURCES + [os.path.join(HERE, "mpcd_oracle.h")]
        if all(os.path.getmtime(s) <= lib_t for s in srcs):
            return LIB_PATH
    return build()


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
