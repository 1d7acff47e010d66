"""Ensembles: independent systems of uneven N held in one context (a forest
of trees, one per system) and stepped by one HIP-graph launch per step.
Every member's forces and every replay are checked against the member in a
context of its own, stepped eagerly with its own time-step, bit for bit,
with the program's own eager GPU work and synchronisations between the
replays.  The members overlap in space, so any interaction that crossed
members would show.  The autotuner returns one of its candidates."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # collected on CPU-only machines but never run there
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_0912_1786_amd import ensemble, inputs, tsph  # noqa: E402

KEYS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "eps", "ax", "ay", "az", "dudt", "rho")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _equal_members(forest, alone, keys, tag):
    for k, sim in enumerate(alone):
        for key in keys:
            a, b = forest.member(k, key), sim.host(key)
            assert np.array_equal(a, b), (tag, k, key, int(np.sum(a != b)))


@pytest.mark.parametrize("precision", [tsph.FP32_BULK, tsph.FP64])
def test_graph_replays_equal_members_alone(precision):
    _say(f"[ensemble] precision={precision}")
    ics = ensemble.ensemble_ics(10, seed=77)
    ens = ensemble.Ensemble(ics, precision=precision)
    prm = ensemble.member_params(precision=precision)
    alone = [tsph.Simulation(ic, prm, want_pot=False) for ic in ics]
    try:
        ens.first_forces()
        for s in alone:
            s.compute_forces()
        torch.cuda.synchronize()
        _equal_members(ens.sim, alone, KEYS, "first forces")
        dts = ens.sim.timestep()
        assert dts.shape == (len(ics),)
        assert np.array_equal(dts, np.array([s.timestep() for s in alone]))
        ens.capture()
        scratch = torch.randn(1 << 20, device="cuda")
        for r in range(3):
            ens.step()
            for s in alone:
                s.device_step()
            torch.cuda.synchronize()
            # the program's own eager work between replays
            scratch = scratch * 0.5 + 1.0
            assert torch.isfinite(scratch.sum()).item()
            torch.cuda.synchronize()
            _equal_members(ens.sim, alone, KEYS, f"replay {r}")
        assert ens.flags() == (0, 0)
        _say(f"    forces and 3 replays equal to the members alone ({ens.n_total} particles)")
    finally:
        ens.close()
        for s in alone:
            s.close()


def _mixed_members():
    """Two-species members of very different sizes: gas fractions between
    a tenth and a half, a member small enough that its root is a walk group
    (and so has no sibling), one below the leaf size of 16."""
    spec = ((3000, 1500, 1), (700, 90, 2), (5000, 800, 3), (60, 30, 4), (12, 6, 5), (1500, 700, 6))
    return [inputs.plummer(n, seed=s, n_gas=g, velocities=True) for n, g, s in spec]


@pytest.mark.parametrize("precision", [tsph.FP32_BULK, tsph.FP64])
def test_two_species_members_equal_alone(precision):
    _say(f"[ensemble] two-species members, precision={precision}")
    ics = _mixed_members()
    big, members = tsph.concat_ics(ics)
    prm = tsph.tsph_default_params(nnei=50.0, precision=precision)
    forest = tsph.Simulation(big, prm, want_pot=True, members=members)
    alone = [tsph.Simulation(ic, prm, want_pot=True) for ic in ics]
    try:
        forest.compute_forces()
        for s in alone:
            s.compute_forces()
        torch.cuda.synchronize()
        _equal_members(forest, alone, KEYS + ("pot",), "forces")
        f_flags = forest.flags()
        a_flags = [s.flags() for s in alone]
        assert f_flags[1] == sum(f[1] for f in a_flags)
        # a KDK step with each member's own time-step, taken on the device
        forest.device_step()
        for s in alone:
            s.device_step()
        torch.cuda.synchronize()
        _equal_members(forest, alone, KEYS + ("pot",), "step")
        # per-member totals (the reductions run in another order: not bitwise)
        d = forest.diagnostics()
        assert d.shape == (len(ics), 9)
        for k, s in enumerate(alone):
            ds = s.diagnostics()
            scale = np.max(np.abs(ds[:3]))
            assert np.allclose(d[k], ds, rtol=1e-12, atol=1e-13 * scale), (k, d[k], ds)
        _say(f"    {len(ics)} members equal alone; flags {f_flags}")
    finally:
        forest.close()
        for s in alone:
            s.close()


def test_member_table_validation():
    ic = inputs.plummer(300, seed=9, n_gas=100)
    prm = tsph.tsph_default_params(max_members=2)
    ctx = tsph.tsph_create(300, prm)
    try:
        with pytest.raises(tsph.TsphError) as e:
            tsph.tsph_set_members(ctx, [0, 100, 200, 300], [10, 10, 10])
        assert e.value.status == tsph.TSPH_ECAPACITY
        for off, gas in (([1, 100, 300], [10, 10]),      # off[0] != 0
                         ([0, 0, 300], [0, 10]),         # an empty member
                         ([0, 100, 300], [101, 10]),     # more gas than particles
                         ([0, 100, 300], [-1, 10])):
            with pytest.raises(tsph.TsphError) as e:
                tsph.tsph_set_members(ctx, off, gas)
            assert e.value.status == tsph.TSPH_EINVAL, (off, gas)
        with pytest.raises(tsph.TsphError) as e:
            tsph.tsph_set_members(ctx, [0, 100, 301], [10, 10])
        assert e.value.status == tsph.TSPH_ECAPACITY
    finally:
        tsph.tsph_destroy(ctx)
    # a state whose sizes are not the members' totals is refused
    sim = tsph.Simulation(ic, prm, members=[(150, 100), (150, 0)])
    try:
        st = sim._state()
        st.n_gas = 50
        with pytest.raises(tsph.TsphError) as e:
            tsph.tsph_compute_forces(sim.ctx, st)
        assert e.value.status == tsph.TSPH_EINVAL
        with pytest.raises(tsph.TsphError):
            sim.carry()
    finally:
        sim.close()


def test_autotuner_picks_a_candidate():
    ics = ensemble.ensemble_ics(6, seed=78)
    tuning = ensemble.autotune(ics, reps=1)
    best = (tuning["leaf"], tuning["group"], tuning["split"])
    assert best in ensemble.CANDIDATES
    times = tuning["ms"]
    assert set(times) == set(ensemble.CANDIDATES)
    assert times[best] == min(times.values())
    assert all(t > 0 for t in times.values())


@pytest.mark.timeout(600)
def test_256_members_equal_alone_on_a_seeded_sample():
    """The full 256-member Evrard ensemble (about 2.3M particles) in one
    context, stepped by graph replays; a seeded sample of 12 members (and
    the smallest and largest) stepped alone equals its forest copy bit for
    bit after the first forces and after two replays."""
    _say("[ensemble] 256 members")
    ics = ensemble.ensemble_ics(256, seed=1000)
    prec = tsph.FP32_BULK
    ens = ensemble.Ensemble(ics, precision=prec)
    prm = ensemble.member_params(precision=prec)
    sizes = np.array([ic["n"] for ic in ics])
    rng = np.random.default_rng(256)
    pick = sorted(set(rng.choice(256, 12, replace=False).tolist()) | {int(sizes.argmin()), int(sizes.argmax())})
    alone = [tsph.Simulation(ics[k], prm, want_pot=False) for k in pick]

    def check(tag):
        for sim, k in zip(alone, pick):
            for key in KEYS:
                a, b = ens.member(k, key), sim.host(key)
                assert np.array_equal(a, b), (tag, k, key, int(np.sum(a != b)))

    try:
        ens.first_forces()
        for s in alone:
            s.compute_forces()
        torch.cuda.synchronize()
        check("first forces")
        ens.capture()
        for r in range(2):
            ens.step()
            for s in alone:
                s.device_step()
            torch.cuda.synchronize()
            check(f"replay {r}")
        assert ens.flags() == (0, 0)
        _say(f"    members {pick} equal alone ({ens.n_total} particles in the forest)")
    finally:
        ens.close()
        for s in alone:
            s.close()
