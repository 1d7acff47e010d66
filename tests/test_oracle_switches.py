"""Pins of the oracle's dissipation switches (Sect. 3.3.1: Balsara limiter
and time-dependent alpha; Sect. 3.3.2: artificial thermal conductivity).

* the velocity curl (h kernel, normalised as the divergence) of a rigid
  rotation on a simple-cubic lattice is exactly 2 omega for interior
  particles, with zero divergence; a homologous flow has zero curl;
* the Balsara factor is |div v| / (|div v| + |curl v| + 1e-4 c/h): ~0 in
  rotation, ~1 in compression;
* the alpha rate is the relaxation -(alpha - alpha_min) / tau with
  tau = h / (0.1 v_sig) (v_sig = 2c at rest) plus the source
  0.75 f max(0, -div v); uniform alpha equal to the fixed one reproduces the
  fixed-alpha forces; the half kicks carry alpha with its rate;
* conduction conserves the total thermal energy exactly, moves heat from hot
  to cold, and its Laplacian of a quadratic u on a lattice is 2 a.
"""
import numpy as np
import pytest

from paper_0912_1786_amd import inputs


def _acc(o):
    return np.stack([o["ax"], o["ay"], o["az"]], 1)


def _lattice(n_side=14, spacing=0.1):
    ic = inputs.cubic_lattice(n_side, spacing=spacing, mass=1.0 / n_side ** 3)
    pos = np.stack([ic["x"], ic["y"], ic["z"]], 1)
    ctr = 0.5 * n_side * spacing
    return ic, pos - ctr


def _interior(pos, h, n_side=14, spacing=0.1):
    half = 0.5 * n_side * spacing
    return np.all(np.abs(pos) < half - 2.2 * h.max(), 1)


def _prm(orc, **kw):
    d = dict(gravity=0, hydro=1, nnei=40, walk_mode=orc.WALK_DIRECT, h_tol=1e-13, leaf_size=8)
    d.update(kw)
    return orc.params(**d)


def test_curl_of_rigid_rotation_and_homologous_flow(orc):
    ic, rel = _lattice()
    omega = np.array([0.3, -0.7, 1.1])
    v = np.cross(omega, rel)
    ir = dict(ic, vx=v[:, 0].copy(), vy=v[:, 1].copy(), vz=v[:, 2].copy())
    o = orc.compute_forces(ir, _prm(orc, balsara=1))
    inner = _interior(rel, o["h"])
    assert inner.sum() > 20
    curl = np.stack([o["curlx"], o["curly"], o["curlz"]], 1)
    assert np.allclose(curl[inner], 2.0 * omega, rtol=1e-10, atol=1e-10)
    assert np.all(np.abs(o["divv"][inner]) < 1e-10)
    assert np.all(o["fbal"][inner] < 1e-8)
    H = 0.4
    vh = -H * rel
    ih = dict(ic, vx=vh[:, 0].copy(), vy=vh[:, 1].copy(), vz=vh[:, 2].copy())
    oh = orc.compute_forces(ih, _prm(orc, balsara=1))
    curl = np.stack([oh["curlx"], oh["curly"], oh["curlz"]], 1)
    assert np.all(np.abs(curl[inner]) < 1e-10)
    assert np.allclose(oh["divv"][inner], -3.0 * H, rtol=1e-10)
    c = np.sqrt(5.0 / 3.0 * (2.0 / 3.0) * ih["u"])
    want = 3 * H / (3 * H + 1e-4 * c / oh["h"])
    assert np.allclose(oh["fbal"][inner], want[inner], rtol=1e-9)


def test_alpha_rate_closed_forms(orc):
    ic, rel = _lattice()
    alpha = np.full(ic["n"], 0.6)
    o = orc.compute_forces(ic, _prm(orc, alpha_switch=1, alpha_min=0.01), alpha=alpha)
    inner = _interior(rel, o["h"])
    c = np.sqrt(5.0 / 3.0 * (2.0 / 3.0) * ic["u"])
    # at rest: v_sig = 2c, no source
    assert np.allclose(o["vsig"][inner], 2 * c[inner], rtol=1e-14)
    want = -(0.6 - 0.01) * 0.1 * 2 * c / o["h"]
    assert np.allclose(o["dalpha"][inner], want[inner], rtol=1e-12)
    # homologous compression: the source 0.75 f (-div v) joins the relaxation
    H = 0.4
    vh = -H * rel
    ih = dict(ic, vx=vh[:, 0].copy(), vy=vh[:, 1].copy(), vz=vh[:, 2].copy())
    oh = orc.compute_forces(ih, _prm(orc, alpha_switch=1, alpha_min=0.01), alpha=alpha)
    tau = oh["h"] / (0.1 * oh["vsig"])
    want = -(0.6 - 0.01) / tau + 0.75 * oh["fbal"] * 3 * H
    assert np.allclose(oh["dalpha"][inner], want[inner], rtol=1e-10)
    assert np.all(oh["dalpha"][inner] > o["dalpha"][inner])


def test_uniform_alpha_equals_fixed_alpha(orc):
    ic = inputs.random_cloud(500, seed=9, masses=(1.0, 5.0), n_gas=500, v_sigma=0.3)
    p = dict(gravity=0, hydro=1, nnei=40, walk_mode=orc.WALK_DIRECT, nbr_mode=orc.NBR_BRUTE, h_tol=1e-13)
    o_fix = orc.compute_forces(ic, orc.params(alpha=0.8, **p))
    o_var = orc.compute_forces(ic, orc.params(alpha=0.8, alpha_switch=1, **p), alpha=np.full(500, 0.8))
    assert np.array_equal(_acc(o_var), _acc(o_fix)) and np.array_equal(o_var["dudt"], o_fix["dudt"])
    # Balsara scales every viscous term by the pair mean of f <= 1
    o_bal = orc.compute_forces(ic, orc.params(alpha=0.8, balsara=1, **p))
    o_inv = orc.compute_forces(ic, orc.params(alpha=0.0, beta=0.0, **p))
    heat_bal = o_bal["dudt"] - o_inv["dudt"]
    heat_fix = o_fix["dudt"] - o_inv["dudt"]
    assert np.all(heat_bal <= heat_fix + 1e-12 * np.abs(heat_fix).max())
    assert np.all(o_bal["fbal"] <= 1.0) and np.all(o_bal["fbal"] >= 0.0)


def test_half_kicks_carry_alpha(orc):
    n = 10
    st = {"n": n, "n_gas": 6, **{k: np.zeros(n) for k in ("x", "y", "z", "vx", "vy", "vz", "u")}}
    alpha = np.linspace(0.05, 1.0, n)
    alpha_u = np.linspace(0.0, 0.3, n)
    dal = np.linspace(-40.0, 5.0, n)
    dalu = np.linspace(-1.0, 1.0, n)
    a0, au0 = alpha.copy(), alpha_u.copy()
    z = np.zeros(n)
    orc.kick_drift(st, 0.01, 0, (z, z, z), z, alphas=dict(alpha=alpha, dalpha=dal, alpha_min=0.01,
                                                          alpha_u=alpha_u, dalpha_u=dalu, alpha_u_min=0.0))
    want = np.maximum(a0 + 0.005 * dal, 0.01)
    wantu = np.maximum(au0 + 0.005 * dalu, 0.0)
    assert np.array_equal(alpha[:6], want[:6]) and np.array_equal(alpha[6:], a0[6:])
    assert np.array_equal(alpha_u[:6], wantu[:6])


def test_conduction(orc):
    ic, rel = _lattice()
    a = 2.5
    u = 1.0 + a * (rel ** 2).sum(1) * 0.0 + a * rel[:, 0] ** 2
    iu = dict(ic, u=u)
    alpha_u = np.full(ic["n"], 0.7)
    on = orc.compute_forces(iu, _prm(orc))
    oc = orc.compute_forces(iu, _prm(orc, conduction=1), alpha_u=alpha_u)
    m = ic["m"]
    dq = oc["dudt"] - on["dudt"]
    # exact conservation of the thermal energy by the conduction terms
    assert abs(np.sum(m * dq)) < 1e-13 * np.sum(m * np.abs(dq))
    assert np.allclose(_acc(oc), _acc(on), rtol=0, atol=0)
    inner = _interior(rel, oc["h"])
    # Brookshaw's Laplacian of u = 1 + a x^2 on the lattice
    assert np.allclose(oc["lapu"][inner], 2 * a, rtol=2e-2), (oc["lapu"][inner].min(), oc["lapu"][inner].max())
    # heat flows down the gradient: the hottest particles cool, the coldest warm
    hot = u >= np.quantile(u, 0.95)
    cold = u <= np.quantile(u, 0.05)
    assert np.all(dq[hot] < 0) and np.all(dq[cold] > 0)
    # the conductivity rate: relaxation to alpha_u_min plus h |lap u| / sqrt(u)
    tau = oc["h"] / (0.1 * oc["vsig"])
    want = -(0.7 - 0.0) / tau + oc["h"] * np.abs(oc["lapu"]) / np.sqrt(u)
    assert np.allclose(oc["dalpha_u"], want, rtol=1e-12)
    # the entropy variable and conduction exclude each other
    with pytest.raises(RuntimeError):
        orc.compute_forces(iu, _prm(orc, conduction=1, entropy=1))
