"""Builds the oracle's C part (test infrastructure only).

Compiles ``mpm_oracle.c`` (and its threaded driver ``mpm_oracle_omp.c``,
OpenMP) with gcc into ``oracle/_build/liboracle_mpm.so``.  Plain -O2 without
fast-math or contraction, so every double operation is performed as written.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
BUILD_DIR = os.path.join(HERE, "_build")
LIB_PATH = os.path.join(BUILD_DIR, "liboracle_mpm.so")
SOURCES = [os.path.join(HERE, "mpm_oracle.c"), os.path.join(HERE, "mpm_oracle_omp.c")]


def build(force=True):
    """Compile the oracle library; with force=False only when missing or stale."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    if not force and os.path.exists(LIB_PATH):
        lib_mtime = os.path.getmtime(LIB_PATH)
        if all(os.path.getmtime(s) <= lib_mtime for s in SOURCES):
            return LIB_PATH
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off",
           "-fno-fast-math", "-fopenmp", "-Wall", "-Wextra", "-o", tmp] + SOURCES + ["-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


if __name__ == "__main__":
    print(build())
