"""Pins of the oracle's gravity (Sect. 2.1 Eqs. Lagrangian, potential,
softphi, dLgravdr, zeta; Sect. 2.2 tree walk, Eq. opcrit; App. B).

* theta = 0 opens every node: the walk is the O(N^2) softened sum.
* theta = 0.5 with quadrupoles stays within 2e-3 relative RMS of it.
* the node expansion's error falls as (l/R)^3 with the quadrupole and as
  (l/R)^2 without (Newtonian direct sum computed here with numpy).
* a Plummer sphere's field and potential match the analytic profile.
* the acceleration, correction terms included, is minus the gradient of the
  softened Lagrangian's potential with self-consistent eps (finite
  differences), and a variant without the correction terms fails that test.
"""
import numpy as np
import pytest
from scipy import integrate

from paper_0912_1786_amd import inputs


def _acc(o):
    return np.stack([o["ax"], o["ay"], o["az"]], 1)


def _relrms(a, b):
    return np.sqrt(np.sum((a - b) ** 2) / np.sum(b ** 2))


@pytest.fixture(scope="module")
def evrard_runs(orc):
    ic = inputs.evrard(4096, seed=1)
    out = {}
    for name, kw in (("direct", dict(walk_mode=orc.WALK_DIRECT)),
                     ("particle", dict(walk_mode=orc.WALK_PARTICLE)),
                     ("group", dict(walk_mode=orc.WALK_GROUP)),
                     ("theta0", dict(walk_mode=orc.WALK_PARTICLE, theta=0.0)),
                     ("theta0g", dict(walk_mode=orc.WALK_GROUP, theta=0.0))):
        out[name] = orc.compute_forces(ic, orc.params(hydro=0, **kw))
    return ic, out


def test_theta_zero_is_direct_sum(evrard_runs):
    ic, o = evrard_runs
    for k in ("theta0", "theta0g"):
        assert _relrms(_acc(o[k]), _acc(o["direct"])) < 1e-13
        assert np.allclose(o[k]["pot"], o["direct"]["pot"], rtol=1e-12)


def test_tree_error_bound(evrard_runs):
    ic, o = evrard_runs
    for k in ("particle", "group"):
        e = _relrms(_acc(o[k]), _acc(o["direct"]))
        assert e < 2e-3, (k, e)
    # the group walk only ever adds interactions, so it is not less accurate
    assert _relrms(_acc(o["group"]), _acc(o["direct"])) <= \
        1.05 * _relrms(_acc(o["particle"]), _acc(o["direct"]))
    assert np.all(o["group"]["cnt_node"] + o["group"]["cnt_pair"] > 0)


def test_momentum_of_the_softened_corrected_sum(orc):
    ic = inputs.random_cloud(700, seed=2, masses=(1.0, 5.0), n_gas=0)
    o = orc.compute_forces(ic, orc.params(walk_mode=orc.WALK_DIRECT, hydro=0, nnei=40))
    ma = ic["m"][:, None] * _acc(o)
    assert np.linalg.norm(ma.sum(0)) < 1e-14 * np.abs(ma).sum()


def _newton(x, y, z, m, p):
    d = p[None, :] - np.stack([x, y, z], 1)
    r = np.linalg.norm(d, axis=1)
    return -(m[:, None] * d / r[:, None] ** 3).sum(0)


@pytest.mark.parametrize("quad,slope", [(True, -3.0), (False, -2.0)])
def test_expansion_error_order(orc, quad, slope):
    rng = np.random.default_rng(11)
    x, y, z = (rng.uniform(-0.5, 0.5, 200) for _ in range(3))
    m = rng.uniform(0.5, 1.5, 200)
    Rs = np.array([8.0, 16.0, 32.0])
    errs = []
    for R in Rs:
        e = []
        for k in range(24):
            v = rng.normal(size=3)
            pnt = R * v / np.linalg.norm(v)
            a, _ = orc.multipole_field(x, y, z, m, pnt, quadrupole=quad)
            ref = _newton(x, y, z, m, pnt)
            e.append(np.linalg.norm(a - ref) / np.linalg.norm(ref))
        errs.append(np.mean(e))
    fit = np.polyfit(np.log(Rs), np.log(errs), 1)[0]
    assert abs(fit - slope) < 0.35, (fit, errs)


def test_plummer_field_and_potential(orc):
    a, c = 1.0, 5.0
    ic = inputs.plummer(1 << 15, seed=3, a=a, rmax_over_a=c, n_gas=0)
    o = orc.compute_forces(ic, orc.params(hydro=0, nnei=50, leaf_size=8, group_size=32))
    pos = np.stack([ic["x"], ic["y"], ic["z"]], 1)
    r = np.linalg.norm(pos, axis=1)
    ar = np.sum(_acc(o) * pos, 1) / r
    xmax = c ** 3 / (c * c + 1) ** 1.5
    Min = lambda s: s ** 3 / (s * s + a * a) ** 1.5 / xmax
    rmax = c * a
    Phi = lambda s: -1.0 / rmax - integrate.quad(lambda t: Min(t) / t ** 2, s, rmax)[0]
    edges = np.array([0.3, 0.5, 0.8, 1.2, 1.8, 2.7, 4.0])
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (r >= lo) & (r < hi)
        rm = r[sel]
        assert np.mean(ar[sel]) == pytest.approx(np.mean(-Min(rm) / rm ** 2), rel=0.02)
        assert np.mean(o["pot"][sel]) == pytest.approx(np.mean([Phi(s) for s in rm[::25]]), rel=0.01)


def _eps_of(orc, ic, prm):
    o = orc.compute_forces(ic, prm)
    assert o["n_noconv"] == 0
    return o["eps"]


@pytest.mark.parametrize("soft_mode,tol", [(0, 1e-7), (2, None)])
def test_force_is_gradient_of_softened_lagrangian(orc, soft_mode, tol):
    """Finite differences of V = (G/2) sum_ij m_i m_j phi(r_ij, eps_i) with
    eps_i = eta n_i^(-1/3) re-solved at every displaced position.  Unequal
    masses (1 : 5).  Without the correction terms the force is not the
    gradient (the test detects the planted omission)."""
    ic = inputs.random_cloud(120, seed=5, masses=(1.0, 5.0), n_gas=0)
    prm = orc.params(walk_mode=orc.WALK_DIRECT, hydro=0, eta_eps=0.9, eta_h=0.9, h_tol=1e-14,
                     soft_mode=soft_mode)
    o = orc.compute_forces(ic, prm)
    acc = _acc(o)
    d = 1e-5
    errs, scale = [], np.abs(acc).mean()
    for i in range(0, 120, 12):
        for k, ax in enumerate("xyz"):
            vals = []
            for s in (+1, -1):
                q = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in ic.items()}
                q[ax][i] += s * d
                eps = _eps_of(orc, q, prm)
                vals.append(orc.potential_energy(q["x"], q["y"], q["z"], q["m"], eps))
            fd = -(vals[0] - vals[1]) / (2 * d) / ic["m"][i]
            errs.append(abs(fd - acc[i, k]) / scale)
    if tol is not None:
        assert max(errs) < tol, max(errs)
    else:
        assert max(errs) > 1e-3, max(errs)


def test_printed_correction_weighting(orc):
    """The printed mass weighting of the correction terms (Eq. dLgravdr with
    xi of Eq. zeta, no masses inside xi): equal to the energy-consistent
    form for equal masses, and not the gradient of the softened Lagrangian
    for unequal masses (1 : 5), where the energy-consistent form is."""
    base = dict(walk_mode=orc.WALK_DIRECT, hydro=0, eta_eps=0.9, eta_h=0.9, h_tol=1e-14)
    eq = inputs.random_cloud(300, seed=8, masses=(1.0, 1.0), n_gas=0)
    a_ec = _acc(orc.compute_forces(eq, orc.params(**base)))
    a_lit = _acc(orc.compute_forces(eq, orc.params(grav_corr_literal=1, **base)))
    assert _relrms(a_lit, a_ec) < 1e-13
    ic = inputs.random_cloud(120, seed=5, masses=(1.0, 5.0), n_gas=0)
    prm = orc.params(grav_corr_literal=1, **base)
    o = orc.compute_forces(ic, prm)
    acc = _acc(o)
    d, scale, errs = 1e-5, np.abs(acc).mean(), []
    for i in range(0, 120, 12):
        for k, ax in enumerate("xyz"):
            vals = []
            for s in (+1, -1):
                q = {kk: (v.copy() if isinstance(v, np.ndarray) else v) for kk, v in ic.items()}
                q[ax][i] += s * d
                eps = _eps_of(orc, q, prm)
                vals.append(orc.potential_energy(q["x"], q["y"], q["z"], q["m"], eps))
            fd = -(vals[0] - vals[1]) / (2 * d) / ic["m"][i]
            errs.append(abs(fd - acc[i, k]) / scale)
    assert max(errs) > 1e-3, max(errs)


def _cluster_and_sink(size, seed):
    """64 particles (masses 1 and 5) inside a ball of radius `size` at the
    origin and one particle at distance 1: the lone particle's softening
    (solved from its neighbour count) reaches the cluster, while the opening
    test passes for the cluster's nodes."""
    rng = np.random.default_rng(seed)
    v = rng.normal(size=(64, 3))
    v *= (rng.uniform(0.0, 1.0, 64) ** (1 / 3) / np.linalg.norm(v, axis=1))[:, None]
    d = rng.normal(size=3)
    pos = np.concatenate([v * size, (d / np.linalg.norm(d))[None, :]])
    m = np.where(np.arange(65) % 2 == 0, 1.0, 5.0) / 65.0
    return {"n": 65, "n_gas": 0, "x": pos[:, 0].copy(), "y": pos[:, 1].copy(), "z": pos[:, 2].copy(),
            "vx": np.zeros(65), "vy": np.zeros(65), "vz": np.zeros(65), "m": m, "u": np.zeros(65)}


@pytest.mark.parametrize("literal", [0, 1])
def test_softened_cells_converge_to_the_pair_sum(orc, literal):
    """A softened cell stands for its particles gathered at their centre of
    mass (Sect. 2.2), correction terms included: as the cluster shrinks, the
    force on the lone particle converges to the exact softened, corrected
    pair sum, linearly or faster in the cluster size."""
    prm = dict(hydro=0, nnei=30, leaf_size=8, theta=0.5, grav_corr_literal=literal, h_tol=1e-13)
    errs = []
    for size in (4e-3, 2e-3, 1e-3, 5e-4):
        e = []
        for seed in range(4):
            ic = _cluster_and_sink(size, seed)
            o = orc.compute_forces(ic, orc.params(soften_cells=1, walk_mode=orc.WALK_PARTICLE, **prm))
            od = orc.compute_forces(ic, orc.params(walk_mode=orc.WALK_DIRECT, **prm))
            assert o["cnt_pair"][64] == 0 and o["cnt_node"][64] > 0  # the cluster came as softened cells
            assert o["eps"][64] > 0.5  # the lone particle's softening reaches the cluster
            a, ad = _acc(o)[64], _acc(od)[64]
            e.append(np.linalg.norm(a - ad) / np.linalg.norm(ad))
        errs.append(np.mean(e))
    errs = np.array(errs)
    assert np.all(errs[1:] < 0.6 * errs[:-1]), errs
    assert errs[-1] < 1e-3, errs


def test_softened_cells_theta_zero_and_accuracy(orc):
    ic = inputs.two_species_field(n_dm=1500, n_gas=1500, n_halo=6, seed=10)
    od = orc.compute_forces(ic, orc.params(walk_mode=orc.WALK_DIRECT, hydro=0, nnei=40))
    o0 = orc.compute_forces(ic, orc.params(walk_mode=orc.WALK_GROUP, theta=0.0, soften_cells=1, hydro=0, nnei=40))
    assert _relrms(_acc(o0), _acc(od)) < 1e-13
    for mode in (orc.WALK_PARTICLE, orc.WALK_GROUP):
        o = orc.compute_forces(ic, orc.params(walk_mode=mode, soften_cells=1, hydro=0, nnei=40))
        on = orc.compute_forces(ic, orc.params(walk_mode=mode, soften_cells=0, hydro=0, nnei=40))
        assert _relrms(_acc(o), _acc(od)) < 2e-3
        # softened cells replace near pairs (fewer pair interactions)
        assert o["cnt_pair"].sum() < on["cnt_pair"].sum()
