"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, -O2, OpenMP over independent sinks, and -ffp-contract=off so that
every predicate rounds once per operation in the stated order.  No
-march=native by default: the built library also runs on the host of the GPU
machine; build(native=True, out=...) makes an -O3 -march=native copy for
timing the oracle on the host that compiles it.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "tsph_oracle.c")
OUT = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, out: str = OUT, native: bool = False) -> str:
    """native: -O3 -march=native, for timing the oracle on the host that
    builds it (the default build also runs on other hosts)."""
    opt = ["-O3", "-march=native"] if native else ["-O2"]
    cmd = ["gcc", *opt, "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11",
           "-D_GNU_SOURCE", "-Wall", "-o", out + ".tmp", SRC, "-lm", "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
