"""Build the oracle's shared library (plain C, FP64, gcc).

Test infrastructure: the oracle is loaded only by the tests, the smoke check
and the CPU-baseline leg of the benchmark.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "fe_oracle.c")
SRC_OMP = os.path.join(HERE, "fe_oracle_omp.c")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liborc.so")
LIB_OMP = os.path.join(OUT_DIR, "liborc_omp.so")  # all-cores build, CPU baseline only


def _compile(src, lib, extra, verbose):
    os.makedirs(OUT_DIR, exist_ok=True)
    tmp = lib + ".tmp"
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-Wall", "-Wno-unused-variable", *extra,
           "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def build(verbose: bool = False) -> str:
    """Compile fe_oracle.c into oracle/_build/liborc.so, single-threaded (the
    parity build), and fe_oracle_omp.c into liborc_omp.so with OpenMP (the
    all-cores CPU baseline).  Always recompiles."""
    _compile(SRC_OMP, LIB_OMP, ["-fopenmp", "-Wno-unknown-pragmas"], verbose)
    return _compile(SRC, LIB, [], verbose)


if __name__ == "__main__":
    print(build(verbose=True))
