"""Build the oracle's C interpolation library with the host C compiler.

Test infrastructure only: the library it produces (``oracle/_interp.so``) is
loaded by the oracle, which only the tests, the smoke check and the
CPU-baseline leg of the benchmark may call.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "interp.c")
LIB = os.path.join(HERE, "_interp.so")


def build(force: bool = True) -> str:
    """Compile interp.c into a shared library; returns its path."""
    if not force and os.path.exists(LIB) and os.path.getmtime(LIB) >= os.path.getmtime(SRC):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", SRC, "-o", tmp, "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
