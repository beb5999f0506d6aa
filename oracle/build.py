"""Compile the oracle's plain C parts with gcc (test infrastructure only)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SO = os.path.join(HERE, "_oracle_jacobi.so")


def build(force: bool = True) -> str:
    if not force and os.path.exists(SO):
        return SO
    tmp = SO + ".tmp"
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-std=c99", "-o", tmp,
           os.path.join(HERE, "jacobi.c"), "-lm"]
    subprocess.check_call(cmd)
    os.replace(tmp, SO)
    return SO


if __name__ == "__main__":
    print(build(force="--if-missing" not in sys.argv))
