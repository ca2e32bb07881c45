"""Builds liboracle.so from fwi2d_oracle.c with gcc (plain -O3, OpenMP).

Run ``python -m oracle.build`` from the repository root, or call ``build()``.
Portable x86-64 code generation: the library is built in one container and
may run on another host.
"""
import os
import subprocess

_HERE = os.path.dirname(os.path.abspath(__file__))


def build(verbose=False):
    src = os.path.join(_HERE, "fwi2d_oracle.c")
    out = os.path.join(_HERE, "liboracle.so")
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wextra",
           "-Wno-unused-parameter", src, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
