"""Compiles the oracle's C source (test infrastructure): oracle/liboracle.so,
single-threaded, and oracle/liboracle_omp.so, the same source with OpenMP
(the parallel CPU baseline)."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def _gcc(out, extra):
    src = os.path.join(HERE, "bolt_oracle.c")
    tmp = out + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-Wall", "-shared", "-fPIC"] + extra + ["-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build() -> str:
    out = _gcc(os.path.join(HERE, "liboracle.so"), ["-Wno-unknown-pragmas"])
    _gcc(os.path.join(HERE, "liboracle_omp.so"), ["-fopenmp"])
    return out


if __name__ == "__main__":
    print(build(), file=sys.stderr)
