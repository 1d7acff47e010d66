"""Ensembles: independent Evrard spheres of uneven N stepped by one HIP-graph
launch per step.  Every replay is checked against the same members stepped
one by one, eagerly, in contexts of their own (bit for bit), with the
program's own eager GPU work and synchronisations between the replays; the
autotuner returns one of its candidates per size class."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only machines but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0912_1786_amd import ensemble, tsph  # noqa: E402

KEYS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "eps", "ax", "ay", "az", "dudt", "rho")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", [tsph.FP32_BULK, tsph.FP64])
def test_graph_replays_equal_members_alone(precision):
    _say(f"[ensemble] precision={precision}")
    ics = ensemble.ensemble_ics(10, seed=77)
    graph = ensemble.Ensemble(ics, precision=precision, streams=4)
    alone = ensemble.Ensemble(ics, precision=precision, streams=1)
    try:
        graph.first_forces()
        alone.first_forces()
        graph.capture()
        scratch = torch.randn(1 << 20, device="cuda")
        for r in range(3):
            graph.step()
            alone.eager_step()
            torch.cuda.synchronize()
            # the program's own eager work between replays
            scratch = scratch * 0.5 + 1.0
            assert torch.isfinite(scratch.sum()).item()
            torch.cuda.synchronize()
            for k, (a, b) in enumerate(zip(graph.members, alone.members)):
                for key in KEYS:
                    assert np.array_equal(a.host(key), b.host(key)), (r, k, key)
        for f in graph.flags():
            assert f == (0, 0)
        _say(f"    3 replays equal to the members stepped alone ({graph.n_total} particles)")
    finally:
        graph.close()
        alone.close()


def test_autotuner_picks_a_candidate():
    ics = ensemble.ensemble_ics(6, seed=78)
    tuning = ensemble.autotune(ics, reps=1)
    assert set(tuning) == {ensemble.size_class(ic["n"]) for ic in ics}
    for c, (leaf, group, times) in tuning.items():
        assert (leaf, group) in ensemble.CANDIDATES
        assert set(times) == set(ensemble.CANDIDATES)
        assert times[(leaf, group)] == min(times.values())
        assert all(t > 0 for t in times.values())
