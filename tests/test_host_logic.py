"""Host-side logic of the ensemble and serving drivers (no GPU): the member
table of a forest, the workload recipes, shell capacity classes and the
request statistics."""
import numpy as np
import pytest

from paper_0912_1786_amd import ensemble, inputs, serve, tsph


def test_concat_ics_member_table():
    ics = [inputs.plummer(n, seed=s, n_gas=g) for n, g, s in ((300, 100, 1), (50, 0, 2), (1000, 1000, 3))]
    big, members = tsph.concat_ics(ics)
    assert members == [(300, 100), (50, 0), (1000, 1000)]
    assert big["n"] == 1350 and big["n_gas"] == 1100
    off = np.cumsum([0] + [m[0] for m in members])
    for k, ic in enumerate(ics):
        for key in ("x", "y", "z", "vx", "vy", "vz", "m", "u"):
            assert np.array_equal(big[key][off[k]:off[k + 1]], ic[key])
        # every member keeps its gas first
        u = big["u"][off[k]:off[k + 1]]
        assert np.all(u[members[k][1]:] == 0.0)


def test_ensemble_recipe():
    ics = ensemble.ensemble_ics(64, seed=1000)
    n = np.array([ic["n"] for ic in ics])
    assert n.min() >= 2 ** 10 - 1 and n.max() <= 2 ** 15 + 1
    assert all(ic["n_gas"] == ic["n"] for ic in ics)
    u0 = np.array([ic["u"][0] for ic in ics])
    assert u0.min() >= 0.02 and u0.max() <= 0.1
    # log-uniform sizes: the mean of log2 N near the middle of [10, 15]
    assert abs(np.mean(np.log2(n)) - 12.5) < 0.5
    # drawn from the seed alone
    again = ensemble.ensemble_ics(3, seed=1000)
    assert [ic["n"] for ic in again] == [ic["n"] for ic in ics[:3]]


def test_shell_capacity_classes():
    assert serve.capacity_class(1) == 4096
    assert serve.capacity_class(4096) == 4096
    assert serve.capacity_class(4097) == 8192
    assert serve.capacity_class(2 ** 20) == 2 ** 20
    assert serve.capacity_class(2 ** 20 + 1) == 2 ** 21
    for n in (5000, 70000, 300000):
        c = serve.capacity_class(n)
        assert c >= n and c < 2 * n and c & (c - 1) == 0


def test_poisson_arrivals_and_summary():
    arr = serve.poisson_arrivals(100.0, 2000, 64, seed=3)
    t = np.array([a for a, _ in arr])
    sims = np.array([s for _, s in arr])
    assert np.all(np.diff(t) > 0)
    assert abs(np.mean(np.diff(t)) - 0.01) < 0.001  # rate 100/s
    assert sims.min() >= 0 and sims.max() <= 63 and len(set(sims.tolist())) > 50
    done = [{"sim": 0, "n": 1000, "arrival": 0.0, "start": 0.0, "end": 0.010},
            {"sim": 1, "n": 3000, "arrival": 0.5, "start": 0.5, "end": 0.520},
            {"sim": 2, "n": 2000, "arrival": 1.0, "start": 1.0, "end": 1.030}]
    s = serve.summarize(done, "x")
    assert s["requests"] == 3
    assert s["p50_ms"] == pytest.approx(20.0)
    assert s["requests_per_s"] == pytest.approx(3 / 1.03, rel=1e-3)
    assert s["particle_steps_per_s"] == pytest.approx(6000 / 1.03, rel=1e-3)
