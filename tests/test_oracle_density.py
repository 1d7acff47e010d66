"""Pins of the oracle's h / eps solve and density sums (Sect. 2.1 Eqs. rho0,
etan, iter; Sect. 3 Eqs. densitySPH, hn, nsum, drhodr; Sect. 3.1 gather and
symmetric neighbour definitions)."""
import json
import os

import numpy as np
import pytest

from paper_0912_1786_amd import inputs

LAT = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "lattice.json")))


def _centre(ic, c):
    pos = np.stack([ic["x"], ic["y"], ic["z"]], 1)
    return int(np.argmin(np.sum((pos - c) ** 2, 1)))


def _lattice_length(eta):
    """Self-consistent h of an interior particle of an infinite simple-cubic
    lattice of unit spacing and unit masses: the lattice sum of the cubic
    spline kernel, n(h) = sum_v w(|v|/h) / (pi h^3), and a bracketed root of
    h^3 n(h) = eta^3 (Sect. 2.1 Eq. etan, Sect. 3 Eq. nsum), written here
    from the definitions, independently of the oracle.  Returns (h, n - 1)."""
    from scipy.optimize import brentq
    g = np.arange(-5, 6)
    v = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3).astype(float)
    r = np.sqrt((v ** 2).sum(1))

    def n_of(h):
        q = r / h
        w = np.where(q < 1, 1 - 1.5 * q ** 2 + 0.75 * q ** 3, np.where(q < 2, 0.25 * (2 - q) ** 3, 0.0))
        return w.sum() / (np.pi * h ** 3)

    h = brentq(lambda h: h ** 3 * n_of(h) - eta ** 3, 0.9, 1.6, xtol=1e-15)
    return h, n_of(h) - 1.0


@pytest.mark.parametrize("eta", ["1.2", "1.2143", "1.1428"])
def test_lattice_self_consistent_length(orc, eta):
    ic = inputs.cubic_lattice(14)
    p = orc.params(eta_h=float(eta), eta_eps=float(eta), gravity=0, hydro=1, h_tol=1e-12)
    out = orc.compute_forces(ic, p)
    c = _centre(ic, 7.0)
    h_ref, excess = _lattice_length(float(eta))
    assert LAT["h_over_delta"][eta] == pytest.approx(h_ref, abs=1e-6)  # the stored fixture agrees
    assert out["h"][c] == pytest.approx(h_ref, abs=1e-10)
    assert out["rho"][c] - 1.0 == pytest.approx(excess, rel=1e-6)
    assert out["rho"][c] - 1.0 == pytest.approx(LAT["rho_excess"][eta], rel=0.1)
    # every interior particle equal to round-off
    pos = np.stack([ic["x"], ic["y"], ic["z"]], 1)
    inner = np.all((pos > 4) & (pos < 10), axis=1)
    assert np.ptp(out["h"][inner]) < 1e-11
    # the relation itself: h^3 n = eta^3 at the solution
    assert out["h"][c] ** 3 * out["nh"][c] == pytest.approx(float(eta) ** 3, rel=1e-12)


def test_bcc_mixed_mass_number_density(orc):
    """Two interpenetrating lattices shifted by half a spacing (the mixed-mass
    density test of Sect. 3): with number-density summation both species see
    the same n, independent of their masses."""
    a = inputs.cubic_lattice(10, spacing=1.0, mass=0.9)
    b = inputs.cubic_lattice(10, spacing=1.0, mass=0.1)
    ic = {k: np.concatenate([a[k], b[k] + (0.5 if k in "xyz" else 0.0)]) for k in
          ("x", "y", "z", "vx", "vy", "vz", "m", "u")}
    ic["n"] = ic["n_gas"] = a["n"] + b["n"]
    deff = 0.5 ** (1.0 / 3.0)  # two particles per unit cell
    p = orc.params(eta_h=1.2, eta_eps=1.2, gravity=0, h_tol=1e-12)
    out = orc.compute_forces(ic, p)
    ia, ib = _centre(ic, 5.0), a["n"] + _centre(b, 5.0)
    assert out["h"][ia] / deff == pytest.approx(out["h"][ib] / deff, rel=1e-10)
    n0 = 2.0
    # n / n0 at the self-consistent length (which sits at h/Delta_eff ~ 1.2)
    assert out["nh"][ia] / n0 == pytest.approx((1.2 / (out["h"][ia] / deff)) ** 3, rel=1e-10)
    assert abs(out["nh"][ia] / n0 - 1.0) < 0.01
    # the mass densities differ only through the neighbours' masses
    assert out["rho"][ia] == pytest.approx(out["rho"][ib], rel=1e-10)


def _numpy_brute(kind, x, y, z, L, n_gas):
    n = x.size
    res = []
    for i in range(n):
        sink = kind == 2 or i < n_gas
        if not sink:
            res.append(np.zeros(0, np.int64))
            continue
        dx, dy, dz = x - x[i], y - y[i], z - z[i]
        r2 = dx * dx + dy * dy
        r2 = r2 + dz * dz
        Lm = L[i] if kind == 0 else np.maximum(L[i], L)
        R = 2.0 * Lm
        ok = r2 < R * R
        if kind != 2:
            ok &= np.arange(n) < n_gas
        if kind != 0:
            ok[i] = False
        res.append(np.nonzero(ok)[0])
    return res


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_neighbour_sets_bit_exact(orc, kind):
    ic = inputs.two_species_field(n_dm=600, n_gas=600, n_halo=4, seed=2)
    p = orc.params(nnei=50)
    out = orc.compute_forces(ic, p)
    L = out["eps"] if kind == 2 else out["h"]
    x, y, z = ic["x"], ic["y"], ic["z"]
    ref = _numpy_brute(kind, x, y, z, L, ic["n_gas"])
    for mode in (orc.NBR_TREE, orc.NBR_BRUTE):
        off, idx = orc.neighbours(kind, x, y, z, L, ic["n_gas"], mode=mode, leaf_size=8)
        for i in range(ic["n"]):
            assert np.array_equal(idx[off[i]:off[i + 1]], ref[i]), (mode, i)


def test_weighted_count_is_nnei(orc):
    """The solved length holds the kernel-weighted count (4 pi/3)(2h)^3 n at
    N_nei (Sect. 2.1, eps-n relation) for every particle of a random field."""
    ic = inputs.random_cloud(8000, seed=3, masses=(1.0, 1.0))
    p = orc.params(nnei=60, gravity=0, h_tol=1e-10)
    out = orc.compute_forces(ic, p)
    h, n = out["h"], out["nh"]
    assert out["n_noconv"] == 0
    assert np.allclose(4 * np.pi / 3 * (2 * h) ** 3 * n, 60.0, rtol=1e-9)


def test_solution_independent_of_guess(orc):
    ic = inputs.evrard(2000, seed=6)
    p = orc.params(gravity=1, hydro=1, h_tol=1e-10)
    cold = orc.compute_forces(ic, p)
    warm = orc.compute_forces(ic, p, h_in=cold["h"] * 0.7, eps_in=cold["eps"] * 1.6)
    assert np.allclose(cold["h"], warm["h"], rtol=1e-11)
    assert np.allclose(cold["eps"], warm["eps"], rtol=1e-11)
    assert np.allclose(cold["rho"], warm["rho"], rtol=1e-10)
    # pure gas with equal etas: eps == h and Upsilon == Omega*
    assert np.allclose(cold["eps"], cold["h"], rtol=1e-11)
    assert np.allclose(cold["ups"], cold["omega"], rtol=1e-9)
    # xi is negative (Sect. 2.1: the correction acts as a negative pressure)
    assert np.all(cold["xi"] < 0)


def test_equal_mass_grad_h_reduction(orc):
    """Equal masses: zeta = m (1 - Omega*), so f_ij = 1/Omega*_i and the
    equations reduce to the standard grad-h form (Sect. 3)."""
    ic = inputs.evrard(1500, seed=7)
    out = orc.compute_forces(ic, orc.params(gravity=0))
    m = ic["m"][0]
    assert np.allclose(out["zeta"], m * (1.0 - out["omega"]), rtol=1e-9, atol=1e-15)


def test_divergence_of_a_homologous_flow_is_exact(orc):
    """With the grad-h normalisation, div v_i = -(1/(n_i Omega*_i)) sum_j
    v_ij . grad_i W_ij reproduces div v = 3H exactly for v = H x, for any
    particle arrangement: sum_j r W'(r) = -(3 n + h dn/dh), and Omega*_i =
    1 + (h/3n) dn/dh cancels the rest.  Holds for the h kernel (gas) and the
    eps kernel (all species)."""
    ic = inputs.two_species_field(n_dm=1500, n_gas=1500, n_halo=4, seed=21)
    H = 0.37
    for k, v in (("x", "vx"), ("y", "vy"), ("z", "vz")):
        ic[v] = H * ic[k]
    p = orc.params(nnei=60, h_tol=1e-12)
    out = orc.compute_forces(ic, p)
    gas = np.arange(ic["n"]) < ic["n_gas"]
    assert np.allclose(out["divv"][gas], 3 * H, rtol=1e-10, atol=0)
    assert np.allclose(out["divv_eps"], 3 * H, rtol=1e-10, atol=0)


def test_length_predictor_is_second_order(orc):
    """Carrying h and eps along a drift with dh/dt = (h/3) div v (continuity
    equation with h n^(1/3) = eta) leaves an error O(dt^2) against the
    re-solved lengths, where the unpredicted lengths are off by O(dt)."""
    ic = inputs.two_species_field(n_dm=1500, n_gas=1500, n_halo=4, seed=22)
    rng = np.random.default_rng(5)
    for v in ("vx", "vy", "vz"):
        ic[v] = rng.normal(0.0, 0.3, ic["n"])
    p = orc.params(nnei=60, h_tol=1e-12)
    o0 = orc.compute_forces(ic, p)
    n_gas = ic["n_gas"]
    zero = np.zeros(ic["n"])
    err = {}
    for dt in (2e-4, 1e-4):
        st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ic.items()}
        ln = {"h": o0["h"].copy(), "eps": o0["eps"].copy(), "divv": o0["divv"], "divv_eps": o0["divv_eps"]}
        orc.kick_drift(st, dt, 0, (zero, zero, zero), zero, None, ln)
        o1 = orc.compute_forces(st, p, h_in=o0["h"], eps_in=o0["eps"])
        rel = lambda a, b: np.abs(a - b) / b
        err[dt] = (np.median(rel(ln["h"][:n_gas], o1["h"][:n_gas])), np.median(rel(o0["h"][:n_gas], o1["h"][:n_gas])),
                   np.median(rel(ln["eps"], o1["eps"])), np.median(rel(o0["eps"], o1["eps"])))
    (ph2, oh2, pe2, oe2), (ph1, oh1, pe1, oe1) = err[2e-4], err[1e-4]
    # predicted: far below the unpredicted error, and quartered when dt halves
    assert ph2 < 0.05 * oh2 and pe2 < 0.05 * oe2
    assert 3.0 < ph2 / ph1 < 5.0 and 3.0 < pe2 / pe1 < 5.0
    # unpredicted: halved when dt halves
    assert 1.7 < oh2 / oh1 < 2.3 and 1.7 < oe2 / oe1 < 2.3
