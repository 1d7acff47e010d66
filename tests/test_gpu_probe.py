"""The machine probes behind the measured roofline denominators: the FMA
chains report the flops they execute and leave their sink untouched; the
stream triad computes a = b + c/2 exactly, over a ragged size."""
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only machines but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0912_1786_amd import tsph  # noqa: E402


def test_probes():
    print("[probe] fma32, fma64, triad n=100003", flush=True)
    sys.stdout.flush()
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    for kind in (tsph.PROBE_FMA32, tsph.PROBE_FMA64):
        assert tsph.tsph_probe(kind, 16, sink.data_ptr()) == 2 * 8 * 16 * 4096 * 256
    torch.cuda.synchronize()
    assert sink.item() == 0.0
    n = 100003
    g = torch.Generator().manual_seed(5)
    b = torch.rand(n, dtype=torch.float64, generator=g)
    c = torch.rand(n, dtype=torch.float64, generator=g)
    a = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    bd, cd = b.cuda(), c.cuda()
    assert tsph.tsph_probe(tsph.PROBE_TRIAD, n, a.data_ptr(), bd.data_ptr(), cd.data_ptr()) == 24 * n
    torch.cuda.synchronize()
    assert torch.equal(a.cpu(), b + 0.5 * c)  # 0.5 c is exact, so one rounding either way
