"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, -O2, no fast-math, OpenMP over pairs.  The oracle links nothing
from the HIP library and includes none of its headers.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ebsd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source built with AddressSanitizer and UndefinedBehaviorSanitizer (host code only);
# loaded instead of LIB when ORACLE_LIB names it and the sanitizer runtimes are preloaded
LIB_SANITIZED = os.path.join(HERE, "liboracle_sanitized.so")


def build(verbose=False, sanitize=False):
    out = LIB_SANITIZED if sanitize else LIB
    extra = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined"] \
        if sanitize else []
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-fno-fast-math",
           "-ffp-contract=off", "-Wall", "-Wno-unused-function"] + extra + [SRC, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
    sys.exit(0)
