"""Build the FP64 CPU oracle (test infrastructure) as oracle/liboracle.so."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose=False, out=LIB, extra=()):
    """Compile dg_oracle.c into out; extra: more gcc flags (the sanitizer test adds
    -fsanitize=address,undefined and builds into a temporary directory)."""
    cmd = ["gcc", "-O3", "-std=gnu11", "-fopenmp", "-fPIC", "-shared",
           "-fno-fast-math", "-ffp-contract=off", *extra,
           "-o", out, os.path.join(HERE, "dg_oracle.c"), "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    return out


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
