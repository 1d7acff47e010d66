"""Pins of the oracle's individual power-of-two time-steps (Sect. 4.2.1).

* every particle in one bin: the block-step run is the global kick-drift-kick
  loop of Sect. 4.1 on the same steps, bit for bit (with the gas, the
  X-SPH drift and the switched dissipation coefficients);
* the energy error of an N-body run with individual steps (direct sums,
  constant softening: the forces are exact gradients of the potential, so the
  error is the integrator's) falls by about four per halving of the
  criterion's eta: second order, as the leapfrog;
* fewer force evaluations than a global run at the same eta, at a comparable
  energy error;
* the wake-up caps the step ratio between SPH neighbours: after every system
  time, each gas neighbour of an active particle is evaluated again within f
  times that particle's criterion step; without the wake-up a point blast on
  a cold lattice breaks this by far;
* the steps are powers of two of the largest step, synchronised: every step
  starts on a multiple of its own length.
"""
import math

import numpy as np
import pytest

from paper_0912_1786_amd import inputs


@pytest.fixture(scope="module")
def blk(orc):
    from oracle import blocksteps
    return blocksteps


def _levels(b):
    return b.L - np.log2(b.t1 - b.t0).astype(int)


def _global_loop(orc, ic, prm, dt_max, L, events, eta_dt=0.1, alpha=None, alpha_u=None):
    """The global kick-drift-kick loop with the common power-of-two step."""
    st = {k: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v) for k, v in ic.items()}
    if alpha is not None:
        st["alpha"] = alpha.copy()
    if alpha_u is not None:
        st["alpha_u"] = alpha_u.copy()
    o = orc.compute_forces(st, prm, alpha=st.get("alpha"), alpha_u=st.get("alpha_u"))
    t = 0
    for _ in range(events):
        dt_c = orc.timestep(prm, st, o, eta_dt)
        lev = L
        for k in range(L + 1):
            if math.ldexp(dt_max, -k) <= dt_c:
                lev = k
                break
        ticks = 1 << (L - lev)
        while t % ticks:
            ticks >>= 1
        dt = math.ldexp(dt_max, ticks.bit_length() - 1 - L)
        pred = {c: st[c].copy() for c in ("vx", "vy", "vz", "u")}
        lengths = {"h": o["h"].copy(), "eps": o["eps"].copy(), "divv": o["divv"], "divv_eps": o["divv_eps"]}
        sw = None
        if alpha is not None or alpha_u is not None:
            z = np.zeros(st["n"])
            sw = dict(alpha=st.get("alpha", z.copy()), dalpha=o["dalpha"] if alpha is not None else z,
                      alpha_min=prm.alpha_min, alpha_u=st.get("alpha_u", z.copy()),
                      dalpha_u=o["dalpha_u"] if alpha_u is not None else z, alpha_u_min=prm.alpha_u_min)
        xs = (o["xsph_x"], o["xsph_y"], o["xsph_z"]) if prm.xsph_eta > 0 else None
        orc.kick_drift(st, dt, 0, (o["ax"], o["ay"], o["az"]), o["dudt"], pred, lengths, xsph=xs, alphas=sw,
                       period=prm.period)
        o = orc.compute_forces(st, prm, h_in=lengths["h"], eps_in=lengths["eps"],
                               vel=(pred["vx"], pred["vy"], pred["vz"]), u=pred["u"],
                               alpha=st.get("alpha"), alpha_u=st.get("alpha_u"))
        if sw is not None:
            sw["dalpha"] = o["dalpha"] if alpha is not None else sw["dalpha"]
            sw["dalpha_u"] = o["dalpha_u"] if alpha_u is not None else sw["dalpha_u"]
        orc.kick_drift(st, dt, 1, (o["ax"], o["ay"], o["az"]), o["dudt"], alphas=sw)
        t = (t + ticks) % (1 << L)
    return st, o


@pytest.mark.parametrize("case", ["plain", "switches", "periodic"])
def test_common_bin_equals_global_loop(orc, blk, case):
    ic = inputs.evrard(300, seed=21, v_sigma=0.05)
    kw = dict(gravity=1, hydro=1, nnei=40, h_tol=1e-12, leaf_size=8)
    if case == "switches":
        kw.update(alpha_switch=1, conduction=1, balsara=1, xsph_eta=0.25, alpha_min=0.05)
    if case == "periodic":
        # the sphere in a box of side 2.5 with a bulk flow across the faces
        L = 2.5
        for k in ("x", "y", "z"):
            ic[k] = np.mod(ic[k] + 1.2, L)
        ic["vx"] = ic["vx"] + 40.0
        kw.update(period=L)
    prm = orc.params(**kw)
    L, events = 6, 5
    o0 = orc.compute_forces(ic, prm)
    dt_max = 4.0 * orc.timestep(prm, ic, o0)
    alpha = np.full(ic["n"], 0.8) if case == "switches" else None
    alpha_u = np.full(ic["n"], 0.1) if case == "switches" else None
    ic_b = dict(ic)
    if alpha is not None:
        ic_b.update(alpha=alpha.copy(), alpha_u=alpha_u.copy())
    b = blk.BlockSteps(ic_b, prm, dt_max, L, common=True)
    assert len(set(_levels(b))) == 1 and _levels(b)[0] > 0
    for _ in range(events):
        act = b.advance()
        assert act.all()
    st, o = _global_loop(orc, ic, prm, dt_max, L, events, alpha=alpha, alpha_u=alpha_u)
    # the block state is mid-step (opening kick done): compare the synchronised
    # velocities and energies, positions and lengths
    for k in ("x", "y", "z"):
        assert np.array_equal(b.st[k], st[k]), k
    assert np.array_equal(b.vs[:, 0], st["vx"]) and np.array_equal(b.vs[:, 2], st["vz"])
    assert np.array_equal(b.us, st["u"])
    assert np.array_equal(b.out["h"], o["h"]) and np.array_equal(b.out["ax"], o["ax"])
    if case == "periodic":
        # wrapped into the box, and the flow has carried particles across x = L
        Lb = kw["period"]
        for k in ("x", "y", "z"):
            assert np.all((b.st[k] >= 0.0) & (b.st[k] < Lb)), k
        assert np.sum(b.st["x"] < ic["x"]) > 10
    if case == "switches":
        # the dissipation coefficients carry the opening kick of the next step
        dt = b.step_dt(b.t1 - b.t0)
        a = np.maximum(st["alpha"] + 0.5 * dt * o["dalpha"], prm.alpha_min)
        assert np.array_equal(b.st["alpha"][:ic["n_gas"]], a[:ic["n_gas"]])
    # a largest step short enough for every criterion: one bin without the
    # common rule, the same run
    if case == "plain":
        b1 = blk.BlockSteps(ic, prm, dt_max / 16, 3)
        assert np.all(_levels(b1) == 0)
        for _ in range(3):
            b1.advance()
        st1, _ = _global_loop(orc, ic, prm, dt_max / 16, 3, 3)
        assert np.array_equal(b1.st["x"], st1["x"]) and np.array_equal(b1.vs[:, 1], st1["vy"])


def _plummer_energy(orc, b):
    s = b.synchronised_state()
    d = orc.diagnostics(s, b.out["pot"])
    return d[0] + d[1] + d[2]


def test_energy_error_is_second_order(orc, blk):
    ic = inputs.plummer(128, seed=5, n_gas=0)
    prm = orc.params(gravity=1, hydro=0, soft_mode=orc.SOFT_CONSTANT, walk_mode=orc.WALK_DIRECT)
    eps = np.full(ic["n"], 0.05)
    errs, evals = [], []
    for eta in (0.1, 0.05, 0.025):
        b = blk.BlockSteps(ic, prm, 0.25, 14, eta_dt=eta, eps_in=eps)
        assert len(set(_levels(b))) >= 3          # a spread of bins
        E0 = _plummer_energy(orc, b)
        worst = 0.0
        for _ in range(8):
            b.run_to_sync()
            worst = max(worst, abs(_plummer_energy(orc, b) - E0) / abs(E0))
            # every step starts on a multiple of its length
            assert np.all(b.t0 % (b.t1 - b.t0) == 0)
        errs.append(worst)
        evals.append(b.sink_evals)
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 6.0 and 3.0 < r2 < 6.0, (errs, r1, r2)
    # the global scheme at the finest eta: every particle in the smallest bin
    g = blk.BlockSteps(ic, prm, 0.25, 14, eta_dt=0.025, eps_in=eps, common=True)
    E0 = _plummer_energy(orc, g)
    gw = 0.0
    for _ in range(8):
        g.run_to_sync()
        gw = max(gw, abs(_plummer_energy(orc, g) - E0) / abs(E0))
    assert g.sink_evals > 1.5 * evals[2]
    assert errs[2] < 5.0 * gw, (errs[2], gw)


def _blast(orc, blk, wake, n_side=10):
    ic = inputs.cubic_lattice(n_side, spacing=1.0 / n_side, mass=1.0 / n_side ** 3)
    ic["u"][:] = 1e-4
    pos = np.stack([ic["x"], ic["y"], ic["z"]], 1)
    c = int(np.argmin(((pos - 0.5) ** 2).sum(1)))
    ic["u"][c] = 100.0
    prm = orc.params(gravity=0, hydro=1, nnei=40, h_tol=1e-12, leaf_size=8)
    return blk.BlockSteps(ic, prm, 0.05, 14, wake=wake)


@pytest.mark.parametrize("wake", [4, 0])
def test_wakeup_caps_neighbour_step_ratio(orc, blk, wake):
    b = _blast(orc, blk, wake)
    worst = 0.0
    for _ in range(40):
        act = b.advance()
        off, nb = orc.neighbours(1, b.st["x"], b.st["y"], b.st["z"], b.out["h"], b.n_gas)
        for i in np.nonzero(act)[0]:
            js = nb[off[i]:off[i + 1]]
            if js.size:
                worst = max(worst, float((b.t1[js] - b.t).max()) / float(b.last_c[i]))
        lens = b.t1 - b.t0
        p2 = (lens & (lens - 1)) == 0               # woken steps are not powers of two
        assert np.all(b.t0[p2] % lens[p2] == 0)
    if wake:
        assert worst <= wake and b.woken > 0, (worst, b.woken)
    else:
        assert worst >= 64, worst
    # only the active particles are evaluated
    assert b.sink_evals < 0.5 * b.n * (b.events + 1)


def test_woken_particle_kick_is_redone(orc, blk):
    """A woken particle's half-kicked velocity equals its synchronised
    velocity plus half the shortened step times its acceleration."""
    b = _blast(orc, blk, 4)
    seen = 0
    for _ in range(20):
        before = b.t1.copy()
        b.advance()
        woken = (b.t1 < before) & (b.t0 < b.t)     # inactive, step cut short
        for j in np.nonzero(woken)[0]:
            dt = b.step_dt([b.t1[j] - b.t0[j]])[0]
            assert b.st["vx"][j] == b.vs[j, 0] + 0.5 * dt * b.out["ax"][j]
            seen += 1
    assert seen > 0
