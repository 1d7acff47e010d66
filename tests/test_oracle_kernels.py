"""Pins of the oracle's kernel functions (Sect. 2.1 Eqs. spline, softforce,
softphi, dphidh; Sect. 3 TC92 gradient; App. A).

Each check comes from outside the oracle's own formulas: exact rational
values at the branch points, the normalisation integral, the Poisson
relation between the force kernel and the density kernel, and finite
differences that tie every derivative to the function it differentiates.
"""
import json
import os

import numpy as np
import pytest
from scipy import integrate

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "kernel_values.json")))


def test_branch_point_values(orc):
    for name, key in (("dphidr", "dphidr"), ("phi", "phi"), ("dphideps", "dphideps")):
        for u, v in GOLD[key].items():
            u = float(u)
            got = orc.kernel(name, [u], [1.0])[0]
            assert got == pytest.approx(v, abs=1e-14), (name, u)
            # the left limit at the branch points agrees too (continuity)
            if u in (1.0, 2.0):
                left = orc.kernel(name, [u - 1e-9], [1.0])[0]
                assert left == pytest.approx(v, abs=1e-7), (name, "left", u)
    for u, v in GOLD["W_times_pi"].items():
        assert np.pi * orc.kernel("W", [float(u)], [1.0])[0] == pytest.approx(v, abs=1e-14)
    for u, v in GOLD["tc92_times_minus_pi"].items():
        assert -np.pi * orc.kernel("tc92", [float(u)], [1.0])[0] == pytest.approx(v, abs=1e-14)


def test_newtonian_beyond_support(orc):
    r = np.linspace(2.0, 9.0, 50)
    for eps in (0.3, 1.0):
        rr = r * eps
        assert np.allclose(orc.kernel("dphidr", rr, eps), 1.0 / rr ** 2, rtol=1e-14)
        assert np.allclose(orc.kernel("phi", rr, eps), -1.0 / rr, rtol=1e-14)
        assert np.all(orc.kernel("dphideps", rr, eps) == 0.0)
        assert np.all(orc.kernel("W", rr, eps) == 0.0)


def test_kernel_normalisation(orc):
    for h in (0.37, 1.0, 2.5):
        val, _ = integrate.quad(lambda r: 4 * np.pi * r * r * orc.kernel("W", [r], [h])[0], 0, 2 * h,
                                points=[h], epsabs=1e-13, epsrel=1e-13)
        assert val == pytest.approx(1.0, abs=1e-12)


def test_poisson_relation(orc):
    """The softened force is that of a unit mass smoothed by W (Sect. 2.1):
    (1/r^2) d/dr (r^2 dphi/dr) = 4 pi W(r, eps)."""
    eps = 0.8
    r = np.linspace(0.05, 2.2, 300) * eps
    d = 1e-6
    f = lambda rr: rr * rr * orc.kernel("dphidr", rr, eps)
    lap = (f(r + d) - f(r - d)) / (2 * d) / r ** 2
    assert np.allclose(lap, 4 * np.pi * orc.kernel("W", r, eps), atol=1e-6)


def test_derivatives_by_finite_differences(orc):
    rng = np.random.default_rng(7)
    r = rng.uniform(0.01, 2.4, 400)
    h = rng.uniform(0.5, 1.5, 400)
    d = 1e-6
    fd_r = lambda name: (orc.kernel(name, r + d, h) - orc.kernel(name, r - d, h)) / (2 * d)
    fd_h = lambda name: (orc.kernel(name, r, h + d) - orc.kernel(name, r, h - d)) / (2 * d)
    assert np.allclose(fd_r("W"), orc.kernel("dWdr", r, h), atol=2e-7)
    assert np.allclose(fd_h("W"), orc.kernel("dWdh", r, h), atol=2e-7)
    assert np.allclose(fd_r("phi"), orc.kernel("dphidr", r, h), atol=2e-7)
    assert np.allclose(fd_h("phi"), orc.kernel("dphideps", r, h), atol=2e-7)


def test_dphideps_outer_branch_sign(orc):
    """The derived outer branch is continuous at u = 1 and vanishes at u = 2;
    the printed '+3/2 u^4' would give 33/10 at u = 1 and 48 at u = 2."""
    u = np.array([1.0, 1.5, 2.0 - 1e-12])
    v = orc.kernel("dphideps", u, 1.0)
    printed = -4 * u ** 2 + 4 * u ** 3 + 1.5 * u ** 4 + 0.2 * u ** 5 + 1.6
    assert v[0] == pytest.approx(0.3, abs=1e-14)
    assert abs(v[2]) < 1e-10
    assert abs(printed[0] - 3.3) < 1e-12 and not np.allclose(v, printed)


def test_tc92_matches_standard_gradient_outside(orc):
    r = np.linspace(1.0, 2.5, 40)
    assert np.allclose(orc.kernel("tc92", r, 1.0), orc.kernel("dWdr", r, 1.0), atol=1e-15)
    r = np.linspace(2 / 3, 1.0, 40)
    assert np.allclose(orc.kernel("tc92", r, 1.0), orc.kernel("dWdr", r, 1.0), atol=1e-15)
    r = np.linspace(0.0, 0.66, 40)
    assert np.allclose(orc.kernel("tc92", r, 1.0), -1.0 / np.pi, atol=1e-15)


def test_eta_nnei_relation(orc):
    """N_nei = (4 pi / 3) (2 eta)^3: eta = 1.2 <-> about 58 and eta = 1.5 <->
    about 113 neighbours (Sect. 2.1 quotes 60 and 110)."""
    nn = lambda eta: 4 * np.pi / 3 * (2 * eta) ** 3
    assert nn(1.2) == pytest.approx(57.9, abs=0.05)
    assert nn(1.5) == pytest.approx(113.1, abs=0.05)
    assert orc.eta_from_nnei(50.0) == pytest.approx(1.142695, abs=1e-6)
    assert orc.eta_from_nnei(60.0) == pytest.approx(1.214295, abs=1e-6)
