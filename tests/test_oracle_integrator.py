"""Pins of the oracle's leapfrog (Sect. 4.1 KDK with predicted velocities)
and of the energy bookkeeping.

* collisionless Evrard sphere with adaptive softening and correction terms
  (a Hamiltonian system once the corrections are in): the energy error of
  KDK scales as dt^2;
* without the correction terms the energy error is larger (Sect. 5,
  collisionless collapse: the corrections reduce the error);
* the full gas + gravity step conserves energy to O(dt^2) as well.
"""
import numpy as np
import pytest

from paper_0912_1786_amd import inputs


def _energy(orc, st, out):
    d = orc.diagnostics(st, out["pot"])
    return d[0] + d[1] + d[2]


def run(orc, ic, prm, dt, nsteps):
    st = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in ic.items()}
    pred = {"vx": st["vx"].copy(), "vy": st["vy"].copy(), "vz": st["vz"].copy(), "u": st["u"].copy()}
    out = orc.compute_forces(st, prm)
    E = [_energy(orc, st, out)]
    for _ in range(nsteps):
        acc = (out["ax"], out["ay"], out["az"])
        orc.kick_drift(st, dt, 0, acc, out["dudt"], pred)
        out = orc.compute_forces(st, prm, h_in=out["h"], eps_in=out["eps"],
                                 vel=(pred["vx"], pred["vy"], pred["vz"]), u=pred["u"])
        orc.kick_drift(st, dt, 1, (out["ax"], out["ay"], out["az"]), out["dudt"])
        E.append(_energy(orc, st, out))
    E = np.array(E)
    return np.max(np.abs(E - E[0])) / abs(E[0])


def test_energy_error_scales_with_dt_squared(orc):
    ic = inputs.evrard(400, seed=3)
    prm = orc.params(hydro=0, walk_mode=orc.WALK_DIRECT, nnei=40, h_tol=1e-12)
    e1 = run(orc, ic, prm, 0.02, 10)
    e2 = run(orc, ic, prm, 0.01, 20)
    assert 3.0 < e1 / e2 < 5.5, (e1, e2)


def test_corrections_reduce_energy_error(orc):
    ic = inputs.evrard(400, seed=4)
    base = dict(hydro=0, walk_mode=orc.WALK_DIRECT, nnei=40, h_tol=1e-12)
    e_corr = run(orc, ic, orc.params(soft_mode=orc.SOFT_ADAPTIVE, **base), 0.01, 20)
    e_none = run(orc, ic, orc.params(soft_mode=orc.SOFT_ADAPTIVE_NOCORR, **base), 0.01, 20)
    # the uncorrected error is secular (independent of dt), the corrected one
    # is the O(dt^2) integration error; the paper reports a factor ~10
    assert e_corr < 0.1 * e_none, (e_corr, e_none)


def test_gas_step_energy_converges(orc):
    ic = inputs.evrard(500, seed=5, v_sigma=0.05)
    prm = orc.params(walk_mode=orc.WALK_DIRECT, nnei=40, h_tol=1e-12)
    e1 = run(orc, ic, prm, 0.01, 6)
    e2 = run(orc, ic, prm, 0.005, 12)
    assert e2 < 0.5 * e1 and e1 < 1e-3, (e1, e2)
