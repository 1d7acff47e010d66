"""Build the HIP library libtsph.so for gfx950 (in-tree).

Each translation unit under csrc/ is compiled with hipcc for gfx950 only, with
packed FP32 instructions disabled, and linked into one shared library that
exports the C ABI of include/tsph.h.  The library carries the identity of the
sources it was built from (tsph_source_id), which the binding checks.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

try:
    from .srcid import source_id
except ImportError:  # run as a script
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from paper_0912_1786_amd.srcid import source_id

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
OUT = os.path.join(HERE, "libtsph.so")
SOURCES = ["tree.hip", "density.hip", "gravity.hip", "sph.hip", "integrate.hip", "blocks.hip", "probe.hip", "abi.hip"]
FLAGS = ["-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC, "-Wall",
         "-Wno-unused-result", "-Wno-unknown-pragmas"]


def _compile(src: str, verbose: bool, sid: str) -> str:
    obj = os.path.join(BUILD, src.replace(".hip", ".o"))
    cmd = ["hipcc", *FLAGS, f'-DTSPH_SOURCE_ID="{sid}"', "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    warn = [l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip()]
    if verbose and warn:
        print("\n".join(warn), flush=True)
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    sid = source_id()
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose, sid), SOURCES))
    cmd = ["hipcc", "-shared", "--offload-arch=gfx950", "-fPIC", "-o", OUT + ".tmp", *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(OUT + ".tmp", OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
