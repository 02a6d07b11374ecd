"""Build the CPU oracle (test infrastructure) into oracle/libmppi_oracle.so."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "mppi_oracle.c")
LIB = os.path.join(HERE, "libmppi_oracle.so")

# -ffp-contract=off: the noise definition is an exact sequence of binary32
# operations; no contraction into fused multiply-adds beyond the explicit ones.
CFLAGS = ["-O2", "-std=c11", "-fno-fast-math", "-ffp-contract=off", "-fPIC",
          "-shared", "-Wall", "-Wextra", "-Wno-unused-parameter"]


def build(verbose: bool = False) -> str:
    tmp = f"{LIB}.{os.getpid()}.tmp"  # concurrent builders each rename their own file
    cmd = ["gcc", *CFLAGS, SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
