"""Pins of the oracle's periodic box (Sect. 4.3): the Ewald correction of
the replicas, the nearest-image pairs of gravity and SPH.

Ewald correction (acceleration per unit mass, displacement x):
* independent of the splitting parameter omega (the real- and Fourier-space
  sums trade terms; a wrong coefficient in either breaks this);
* the replicas and the neutralising background give (4 pi / 3) x / L^3 near
  the origin (the lattice field is isotropic to second order);
* where the periodic force vanishes by symmetry (half-way to a replica, the
  face and cube centres) the correction cancels the direct term, x/|x|^3;
* odd in its own coordinate, even in the others; the tabulated form equals
  the sums on its grid and stays within a stated bound between the nodes.
Gravity and SPH in the box:
* a perfect cubic lattice feels no force (direct sums) and every particle
  gets the same density; a lattice shifted across the faces gives the same;
* forces are invariant under a translation modulo L (direct sums), and the
  total momentum rate vanishes;
* the neighbour sets equal a brute-force nearest-image search.
"""
import math

import numpy as np
import pytest

from paper_0912_1786_amd import inputs


def _exact(orc, x, L, w=None):
    return orc.ewald(x[0], x[1], x[2], L, 2.0 / L if w is None else w)


def test_ewald_independent_of_omega(orc):
    L = 1.7
    rng = np.random.default_rng(1)
    for x in rng.uniform(-0.5 * L, 0.5 * L, (20, 3)):
        a = _exact(orc, x, L)
        for wl in (1.5, 3.0):
            b = _exact(orc, x, L, wl / L)
            assert np.allclose(a, b, rtol=1e-9, atol=1e-11 / L ** 2), (x, a, b)


def test_ewald_closed_forms(orc):
    L = 2.0
    # near the origin: (4 pi / 3) x / L^3
    for x in ([1e-3, 0.0, 0.0], [3e-4, -2e-4, 5e-4]):
        x = np.array(x) * L
        want = 4.0 * math.pi / 3.0 * x / L ** 3
        assert np.allclose(_exact(orc, x, L), want, rtol=1e-5, atol=1e-12 * np.abs(want).max()), x
    # zero periodic force: the correction is the direct term x/|x|^3
    for x in ([0.5, 0, 0], [0.5, 0.5, 0], [0.5, 0.5, 0.5], [0, -0.5, 0.5]):
        x = np.array(x, dtype=float) * L
        want = x / np.linalg.norm(x) ** 3
        assert np.allclose(_exact(orc, x, L), want, rtol=1e-10, atol=1e-12), x
    # symmetry
    x = np.array([0.3, -0.1, 0.2]) * L
    a = _exact(orc, x, L)
    b = _exact(orc, x * np.array([-1, 1, 1]), L)
    assert np.allclose(b, a * np.array([-1, 1, 1]), rtol=1e-12, atol=1e-14)
    assert np.all(_exact(orc, np.zeros(3), L) == 0.0)


def test_ewald_table(orc):
    L = 1.0
    step = 0.5 * L / 32
    rng = np.random.default_rng(2)
    # on the grid: the sums themselves
    for ijk in rng.integers(0, 33, (20, 3)):
        x = ijk * step * rng.choice([-1.0, 1.0], 3)
        assert np.allclose(orc.ewald(*x, L), _exact(orc, x, L), rtol=1e-12, atol=1e-12)
    # between the nodes: trilinear interpolation of a smooth field; the error
    # is far below the direct force at these distances
    worst = 0.0
    for x in rng.uniform(-0.5, 0.5, (400, 3)) * L:
        e = np.abs(orc.ewald(*x, L) - _exact(orc, x, L)).max()
        worst = max(worst, e)
    assert worst < 2e-3 * 4.0 / L ** 2, worst


def _lattice(n_side, L):
    ic = inputs.cubic_lattice(n_side, spacing=L / n_side, mass=1.0 / n_side ** 3)
    for k in ("x", "y", "z"):
        ic[k] = ic[k] + 0.5 * L / n_side  # cell centres, inside [0, L)
    return ic


def _prm(orc, L, **kw):
    d = dict(gravity=1, hydro=1, nnei=40, h_tol=1e-12, leaf_size=8, period=L, walk_mode=orc.WALK_DIRECT,
             soft_mode=orc.SOFT_CONSTANT)
    d.update(kw)
    return orc.params(**d)


def _acc(o):
    return np.stack([o["ax"], o["ay"], o["az"]], 1)


def test_lattice_feels_no_force_and_uniform_density(orc):
    L, ns = 1.0, 8
    ic = _lattice(ns, L)
    eps = np.full(ic["n"], 0.3 * L / ns)
    o = orc.compute_forces(ic, _prm(orc, L), eps_in=eps)
    scale = ic["m"][0] / (L / ns) ** 2
    assert np.abs(_acc(o)).max() < 1e-10 * scale
    assert np.allclose(o["rho"], o["rho"][0], rtol=1e-12)
    assert np.allclose(o["h"], o["h"][0], rtol=1e-12)
    # shifted across the faces
    sh = dict(ic)
    shift = np.array([0.37, -0.21, 0.55]) * L
    for k, d in zip(("x", "y", "z"), shift):
        sh[k] = np.mod(ic[k] + d, L)
    o2 = orc.compute_forces(sh, _prm(orc, L), eps_in=eps)
    assert np.abs(_acc(o2)).max() < 1e-10 * scale
    assert np.allclose(o2["rho"], o["rho"][0], rtol=1e-12)
    # the open box is not uniform: the periodic images matter
    o3 = orc.compute_forces(ic, _prm(orc, 0.0), eps_in=eps)
    assert np.abs(_acc(o3)).max() > 1e-2 * scale


def test_translation_invariance_and_momentum(orc):
    L = 2.0
    ic = inputs.random_cloud(400, seed=11, masses=(1.0, 3.0), n_gas=250, v_sigma=0.2)
    for k in ("x", "y", "z"):
        ic[k] = np.mod(ic[k] * 1.3, L)
    prm = _prm(orc, L, soft_mode=orc.SOFT_ADAPTIVE)
    o = orc.compute_forces(ic, prm)
    m = ic["m"]
    ma = m[:, None] * _acc(o)
    assert np.linalg.norm(ma.sum(0)) < 1e-12 * np.abs(ma).sum()
    sh = dict(ic)
    for k, d in zip(("x", "y", "z"), (0.71, 1.33, -0.4)):
        sh[k] = np.mod(ic[k] + d, L)
    o2 = orc.compute_forces(sh, prm)
    assert np.allclose(_acc(o2), _acc(o), rtol=1e-8, atol=1e-10 * np.abs(_acc(o)).max())
    assert np.allclose(o2["dudt"], o["dudt"], rtol=1e-8, atol=1e-10 * np.abs(o["dudt"]).max())
    assert np.allclose(o2["h"], o["h"], rtol=1e-10)


def test_two_body_force(orc):
    L = 1.0
    ic = {"n": 2, "n_gas": 0, "x": np.array([0.1, 0.85]), "y": np.array([0.2, 0.3]), "z": np.array([0.9, 0.05]),
          "vx": np.zeros(2), "vy": np.zeros(2), "vz": np.zeros(2), "m": np.array([1.0, 2.0]), "u": np.zeros(2)}
    o = orc.compute_forces(ic, _prm(orc, L, hydro=0), eps_in=np.full(2, 1e-3))
    d = np.array([ic["x"][0] - ic["x"][1], ic["y"][0] - ic["y"][1], ic["z"][0] - ic["z"][1]])
    d = d - L * np.round(d / L)
    want = 2.0 * (-d / np.linalg.norm(d) ** 3 + orc.ewald(*d, L))
    assert np.allclose(_acc(o)[0], want, rtol=1e-12)
    exact = 2.0 * (-d / np.linalg.norm(d) ** 3 + _exact(orc, d, L))
    assert np.allclose(_acc(o)[0], exact, rtol=5e-3)


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_periodic_neighbours_brute_force(orc, kind):
    L = 1.0
    ic = inputs.random_cloud(300, seed=12, masses=(1.0, 2.0), n_gas=200, v_sigma=0.0)
    x, y, z = (np.mod(ic[k], L) for k in ("x", "y", "z"))
    n, ng = ic["n"], ic["n_gas"]
    length = np.random.default_rng(3).uniform(0.04, 0.12, n)
    off, idx = orc.neighbours(kind, x, y, z, length, ng, period=L)
    pos = np.stack([x, y, z], 1)
    for i in range(n):
        if kind != 2 and i >= ng:
            assert off[i + 1] == off[i]
            continue
        d = pos - pos[i]
        d -= L * np.round(d / L)
        r2 = (d ** 2).sum(1)
        R = 2 * length[i] if kind == 0 else 2 * np.maximum(length[i], length)
        ok = r2 < R ** 2
        if kind != 2:
            ok &= np.arange(n) < ng
        if kind != 0:
            ok[i] = False
        assert np.array_equal(idx[off[i]:off[i + 1]], np.nonzero(ok)[0]), i


@pytest.mark.parametrize("walk", ["group", "particle"])
def test_periodic_tree_walk_close_to_direct(orc, walk):
    """The periodic tree walks (nearest-image opening tests, multipoles and
    the correction per accepted node) approximate the periodic direct sums
    as the open walks do the open ones."""
    L = 1.0
    ic = inputs.random_cloud(1500, seed=13, masses=(1.0, 3.0), n_gas=0, v_sigma=0.0)
    for k in ("x", "y", "z"):
        ic[k] = np.mod(ic[k] * 0.8, L)
    mode = orc.WALK_GROUP if walk == "group" else orc.WALK_PARTICLE
    kw = dict(hydro=0, soft_mode=orc.SOFT_ADAPTIVE)
    o_t = orc.compute_forces(ic, _prm(orc, L, walk_mode=mode, **kw))
    o_d = orc.compute_forces(ic, _prm(orc, L, **kw))
    a_t, a_d = _acc(o_t), _acc(o_d)
    err = np.sqrt(((a_t - a_d) ** 2).sum(1).mean() / (a_d ** 2).sum(1).mean())
    assert err < 3e-3, err
    # the replicas matter at this size
    o_o = orc.compute_forces(ic, _prm(orc, 0.0, **kw))
    err_o = np.sqrt(((_acc(o_o) - a_d) ** 2).sum(1).mean() / (a_d ** 2).sum(1).mean())
    assert err_o > 10 * err, (err_o, err)
