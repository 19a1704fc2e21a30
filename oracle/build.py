"""Build the CPU oracle shared library (oracle/liboracle.so) with gcc."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = LIB, defines=(), extra=()) -> str:
    """Compiles oracle.c into the shared library `out` (the default path is the
    one the oracle package loads).  `defines` (NAME=VALUE) and `extra` compiler
    flags serve the tests only: mutants of the oracle and sanitizer builds go to
    other paths."""
    cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=gnu11", "-Wall", "-Wextra",
           "-Wno-unused-parameter", *[f"-D{d}" for d in defines], *extra, "-o", out + ".tmp",
           os.path.join(HERE, "oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
