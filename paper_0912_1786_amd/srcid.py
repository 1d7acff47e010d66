"""Identity of the library sources: a SHA-256 over the HIP sources and the
C header, compiled into libtsph.so (tsph_source_id) so that the binding can
refuse a library built from other sources than the ones beside it."""
import hashlib
import os

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def source_files():
    csrc = os.path.join(HERE, "csrc")
    names = sorted(f for f in os.listdir(csrc) if f.endswith((".hip", ".h")))
    return [os.path.join(csrc, f) for f in names] + [os.path.join(ROOT, "include", "tsph.h")]


def source_id() -> str:
    h = hashlib.sha256()
    for path in source_files():
        h.update(os.path.basename(path).encode())
        h.update(b"\0")
        with open(path, "rb") as f:
            h.update(f.read())
        h.update(b"\0")
    return h.hexdigest()[:16]
