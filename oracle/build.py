"""Builds the oracle's shared library (plain C, FP64, OpenMP) with gcc."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dpcg_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
# the same source built with AddressSanitizer and UndefinedBehaviorSanitizer, loaded in
# place of LIB when ORACLE_SANITIZED=1 (the host process must preload the ASan runtime)
LIB_SAN = os.path.join(HERE, "liboracle_san.so")
SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
             "-fno-sanitize-recover=undefined"]


def build(verbose=False, sanitize=False):
    out = LIB_SAN if sanitize else LIB
    opt = SAN_FLAGS if sanitize else ["-O2"]
    cmd = ["gcc"] + opt + ["-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
                           "-o", out + ".tmp", SRC, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    import sys
    print(build(verbose=True, sanitize="--sanitize" in sys.argv))
