"""Serving: single-step requests for resident simulations of different N
and species mix, run concurrently on several streams under an HBM budget
small enough to force evictions.  Each simulation's state after its served
steps equals the same number of steps run alone, bit for bit."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only machines but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0912_1786_amd import serve, tsph  # noqa: E402

KEYS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "eps", "ax", "ay", "az", "dudt", "rho")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_served_results_equal_alone():
    ics = serve.population(6, seed=4000, lo_log2=12.0, hi_log2=15.0)
    probe = serve.Server(ics, streams=4)
    total = sum(r.bytes() for r in probe.res)
    probe.close()
    srv = serve.Server(ics, streams=4, hbm_budget=int(0.45 * total))
    try:
        arr = serve.poisson_arrivals(2000.0, 40, len(ics), seed=5)
        done = srv.run(arr)
        assert len(done) == 40
        s = serve.summarize(done, "test")
        _say(f"    {s}; evictions {srv.evictions}, admissions {srv.admissions}")
        assert srv.evictions > 0
        for sid, f in srv.flags():
            assert f == (0, 0), sid
        for r in srv.res:
            if r.steps == 0:
                continue
            state = {k: r.host(k) for k in KEYS}
            alone = tsph.Simulation(r.ic, r.params, want_pot=False)
            try:
                alone.compute_forces()
                for _ in range(r.steps):
                    alone.device_step()
                torch.cuda.synchronize()
                for k in KEYS:
                    assert np.array_equal(state[k], alone.host(k)), (r.sid, r.steps, k)
            finally:
                alone.close()
    finally:
        srv.close()


def test_population_recipe():
    ics = serve.population(16, seed=4100)
    for ic in ics:
        assert 2 ** 12 - 1 <= ic["n"] <= 2 ** 20 + 1
        assert ic["n_gas"] == 0 or 64 <= ic["n_gas"] <= ic["n"]
        assert np.allclose(ic["m"], ic["m"][0])
    assert {ic["kind"] for ic in ics} == {"evrard", "plummer"}
