"""Pins of the oracle's time-step rule (Sect. 4.2) and diagnostics.

Time-step: particles built so that each criterion of Sect. 4.2 decides in
turn, with values worked out by hand from the printed criteria:
  dt_acc = eta sqrt(min(eps, h) / |a|),
  dt_C   = eta h / (h |div v| + c + 1.2 (alpha c + beta max|mu|)),
  dt_u   = eta |u / (du/dt)|,
and the global step is the smallest over particles and criteria.

Diagnostics: a rigid rotation about the centre of mass plus a uniform drift
has closed forms that share nothing with a sum of cross products:
P = M V, L = M R x V + I omega with the inertia tensor
I = sum m (|r|^2 1 - r r^T) about the centre of mass, and
E_kin = M |V|^2 / 2 + omega . I omega / 2.
"""
import numpy as np
import pytest


def _one(orc, prm, *, a=(0.0, 0.0, 0.0), h=1.0, eps=1.0, u=0.9, dudt=0.0, divv=0.0, maxmu=0.0, gas=True):
    """The global step of a single particle with these values."""
    st = {"n": 1, "n_gas": 1 if gas else 0, "vx": np.zeros(1), "vy": np.zeros(1), "vz": np.zeros(1),
          "u": np.array([u])}
    out = {"h": np.array([h]), "eps": np.array([eps]), "ax": np.array([a[0]]), "ay": np.array([a[1]]),
           "az": np.array([a[2]]), "dudt": np.array([dudt]), "divv": np.array([divv]),
           "maxmu": np.array([maxmu])}
    return orc.timestep(prm, st, out, eta_dt=0.1)


def test_acceleration_criterion(orc):
    prm = orc.params(hydro=0)
    # |a| = 5 (3-4-0), min(eps, h) = 0.2: dt = 0.1 sqrt(0.2 / 5) = 0.02
    assert _one(orc, prm, a=(3.0, 4.0, 0.0), eps=0.2, h=7.0, gas=False) == pytest.approx(0.02, rel=1e-15)
    # a gas particle takes the smaller of its two lengths
    prm_g = orc.params(hydro=0)
    assert _one(orc, prm_g, a=(0.0, 0.0, 8.0), eps=0.5, h=0.02, u=0.0) == pytest.approx(0.1 * 0.05, rel=1e-15)


def test_courant_criterion_with_viscosity_term(orc):
    prm = orc.params(gamma=5.0 / 3.0, alpha=1.0, beta=2.0)
    # u = 0.9 gives c^2 = gamma (gamma - 1) u = 1, so c = 1.  At rest, with no
    # divergence and no approaching pair: den = c + 1.2 alpha c = 2.2
    assert _one(orc, prm, h=1.0, u=0.9) == pytest.approx(0.1 / 2.2, rel=1e-14)
    # with div v = -0.5 (|div v| h = 0.5 for h = 1) and max|mu| = 0.25:
    # den = 0.5 + 1 + 1.2 (1 + 2 x 0.25) = 3.3
    assert _one(orc, prm, h=1.0, u=0.9, divv=-0.5, maxmu=0.25) == pytest.approx(0.1 / 3.3, rel=1e-14)
    # the criterion scales with h at fixed c and mu (h / (h|div v| + ...))
    assert _one(orc, prm, h=2.0, u=0.9) == pytest.approx(0.2 / 2.2, rel=1e-14)
    # alpha and beta enter only through 1.2 (alpha c + beta max|mu|)
    prm2 = orc.params(gamma=5.0 / 3.0, alpha=0.5, beta=4.0)
    assert _one(orc, prm2, h=1.0, u=0.9, maxmu=0.25) == pytest.approx(0.1 / (1.0 + 1.2 * (0.5 + 1.0)), rel=1e-14)


def test_thermal_criterion(orc):
    prm = orc.params()
    # u = 0.9, du/dt = -90: dt_u = 0.1 x 0.01 = 1e-3, below the Courant 0.1/2.2
    assert _one(orc, prm, h=1.0, u=0.9, dudt=-90.0) == pytest.approx(1e-3, rel=1e-14)
    # du/dt = 0 imposes nothing
    assert _one(orc, prm, h=1.0, u=0.9, dudt=0.0) == pytest.approx(0.1 / 2.2, rel=1e-14)


def test_global_step_is_the_smallest_over_particles_and_criteria(orc):
    prm = orc.params()
    # four particles, each decided by another criterion; the last is dark
    # matter (only the acceleration criterion applies to it)
    st = {"n": 4, "n_gas": 3, "vx": np.zeros(4), "vy": np.zeros(4), "vz": np.zeros(4),
          "u": np.array([0.9, 0.9, 0.9, 0.0])}
    out = {"h": np.array([1.0, 1.0, 1.0, 0.0]), "eps": np.array([1.0, 1.0, 1.0, 0.2]),
           "ax": np.array([0.0, 0.0, 0.0, 3.0]), "ay": np.array([0.0, 0.0, 0.0, 4.0]), "az": np.zeros(4),
           "dudt": np.array([0.0, -90.0, 0.0, 0.0]), "divv": np.array([0.0, 0.0, -0.5, 0.0]),
           "maxmu": np.array([0.0, 0.0, 0.25, 0.0])}
    want = {0: 0.1 / 2.2, 1: 1e-3, 2: 0.1 / 3.3, 3: 0.02}
    assert orc.timestep(prm, st, out, eta_dt=0.1) == pytest.approx(min(want.values()), rel=1e-14)
    # remove the binding particle's criterion: the next one decides
    out["dudt"][1] = 0.0
    assert orc.timestep(prm, st, out, eta_dt=0.1) == pytest.approx(0.02, rel=1e-14)
    out["ax"][3] = out["ay"][3] = 0.0
    assert orc.timestep(prm, st, out, eta_dt=0.1) == pytest.approx(0.1 / 3.3, rel=1e-14)
    # eta_dt scales every criterion
    assert orc.timestep(prm, st, out, eta_dt=0.3) == pytest.approx(0.3 / 3.3, rel=1e-14)


def test_rigid_rotation_diagnostics(orc):
    rng = np.random.default_rng(5)
    n = 257
    r = rng.normal(size=(n, 3)) * np.array([1.0, 0.6, 0.3])
    m = rng.uniform(0.5, 2.0, n)
    R = np.array([0.3, -1.2, 2.0])  # centre of mass after the shift below
    com = (m[:, None] * r).sum(0) / m.sum()
    x = r - com + R
    omega = np.array([0.7, -0.4, 1.3])
    V = np.array([0.05, 0.2, -0.1])
    v = np.cross(omega, x - R) + V
    st = {"n": n, "n_gas": 100, "x": x[:, 0], "y": x[:, 1], "z": x[:, 2], "vx": v[:, 0], "vy": v[:, 1],
          "vz": v[:, 2], "m": m, "u": np.full(n, 0.25)}
    pot = rng.normal(size=n)
    d = orc.diagnostics(st, pot)
    M = m.sum()
    s = x - R
    inertia = (m[:, None, None] * ((s * s).sum(1)[:, None, None] * np.eye(3) - s[:, :, None] * s[:, None, :])).sum(0)
    assert np.allclose(d[3:6], M * V, rtol=1e-12, atol=1e-12)
    assert np.allclose(d[6:9], M * np.cross(R, V) + inertia @ omega, rtol=1e-11, atol=1e-11)
    assert d[0] == pytest.approx(0.5 * M * V @ V + 0.5 * omega @ inertia @ omega, rel=1e-12)
    assert d[1] == pytest.approx(0.25 * m[:100].sum(), rel=1e-14)
    assert d[2] == pytest.approx(0.5 * (m * pot).sum(), rel=1e-12)
