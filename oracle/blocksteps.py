"""Individual power-of-two time-steps (Sect. 4.2.1) on the oracle's forces.

TEST INFRASTRUCTURE ONLY, like the rest of this package: the tests, the
smoke check and the benchmark's CPU-baseline leg use it; the HIP package
never imports it.

What is computed (the paper's recipe, with the readings stated):

* Time runs in integer ticks: the largest step dt_max is 2^L ticks of
  dt_max / 2^L.  Particle i advances with dt_max / 2^n_i, n_i in [0, L],
  the largest such step not above its criterion of Sect. 4.2 (the printed
  inequality is read with the step at most the criterion: the smallest n_i
  whose step does not exceed it; n_i = L where even that is too long).
* A particle may only take a longer step where the new bin is synchronised
  with the current time: the step taken is the largest power of two not above
  the criterion's that divides the current tick.
* The next system time is the earliest step end; the particles whose step
  ends there are active.  Each step is a kick-drift-kick leapfrog (Sect.
  4.1) of the particle's own length: the opening half kick at its start, the
  drift of every particle to each system time with its half-kicked
  velocity, the closing half kick at its end with the acceleration computed
  there.
* Forces (gravity and the SPH sums) are evaluated for the active particles
  only; the others keep their accelerations and rates.  The velocities and
  internal energies that every particle lends to the forces are the
  predicted ones of Sect. 4.1: v_n + a_n (t - t_n) from the particle's last
  synchronised state.  Reading: the lengths and densities of all gas
  particles are solved again at every system time (the paper solves them
  for the active ones only and predicts the rest); the pair terms of the
  active particles then see their neighbours at the current time.
* Wake-up: after the active particles have chosen their criterion steps c_i,
  an active gas particle takes at most f times (f = 4 by default, the
  paper's 4-8) the shortest current step among its SPH neighbours
  (r_ij < 2 max(h_i, h_j)); an inactive gas particle whose ongoing step is
  longer than f times the shortest criterion step w of its active
  neighbours ends its step early, at the current time plus w, with its
  opening half kick redone for the shortened step (its drift so far is kept,
  which is why the paper notes that a woken particle does not conserve
  energy and momentum exactly).
* ``common=True`` is the global scheme of Sect. 4.2: every particle takes the
  bin of the smallest criterion.

With all particles in one bin the arithmetic is that of the global
kick-drift-kick loop on the same step, operation for operation.
"""
from __future__ import annotations

import math

import numpy as np

from . import oracle as O

# force outputs kept per particle from its last evaluation as a sink
_SINK_FIELDS = ("ax", "ay", "az", "pot", "dudt", "maxmu", "xsph_x", "xsph_y", "xsph_z", "vsig", "dalpha",
                "dalpha_u", "curlx", "curly", "curlz", "fbal", "lapu", "cnt_node", "cnt_pair", "cnt_sph",
                "cnt_soft")


def _pow2_floor(k: np.ndarray) -> np.ndarray:
    """Largest power of two <= k (k >= 1, integers)."""
    k = np.asarray(k, np.int64)
    out = np.ones_like(k)
    for i in range(k.size):
        out.flat[i] = 1 << (int(k.flat[i]).bit_length() - 1)
    return out


class BlockSteps:
    """A run with individual time-steps.  ``st`` is the state dict (x, y, z,
    vx, vy, vz, u, m, n, n_gas; alpha / alpha_u with the switches); ``t``
    the system time in ticks; ``t0``/``t1`` each particle's step start and
    end (ticks); ``out`` the merged outputs of the last evaluations."""

    def __init__(self, ic: dict, prm, dt_max: float, max_level: int, eta_dt: float = 0.1, wake: int = 4,
                 common: bool = False, eps_in=None):
        assert 0 <= max_level <= 40 and dt_max > 0
        assert wake == 0 or (wake & (wake - 1)) == 0, "the wake-up factor is a power of two (0: off)"
        self.prm, self.eta_dt, self.wake, self.common = prm, eta_dt, int(wake), bool(common)
        self.L = int(max_level)
        self.T = 1 << self.L
        self.dt_max = float(dt_max)
        self.dtu = math.ldexp(self.dt_max, -self.L)
        n = int(ic["n"])
        self.n, self.n_gas = n, int(ic["n_gas"])
        self.st = {k: (np.array(v, dtype=np.float64) if isinstance(v, np.ndarray) else v) for k, v in ic.items()}
        if prm.alpha_switch and "alpha" not in self.st:
            self.st["alpha"] = np.full(n, prm.alpha)
        if prm.conduction and "alpha_u" not in self.st:
            self.st["alpha_u"] = np.zeros(n)
        self.t = 0
        self.t0 = np.zeros(n, np.int64)
        self.t1 = np.zeros(n, np.int64)
        self.vs = np.stack([self.st["vx"], self.st["vy"], self.st["vz"]], 1).copy()
        self.us = self.st["u"].copy()
        self.h = None
        self.eps = None if eps_in is None else np.array(eps_in, dtype=np.float64)
        self.out = None
        self.sink_evals = 0       # number of sink force evaluations (work)
        self.events = 0
        self.woken = 0
        self.last_active = None   # active mask and criterion steps of the last event
        self.last_c = None
        # first evaluation with every particle active
        self._evaluate(np.ones(n, bool))
        self._start_steps(np.ones(n, bool))

    # ---- helpers ---------------------------------------------------------
    def step_dt(self, ticks) -> np.ndarray:
        """dt of steps of the given lengths in ticks; powers of two are exact."""
        ticks = np.asarray(ticks, np.int64)
        return np.array([math.ldexp(self.dt_max, int(k).bit_length() - 1 - self.L)
                         if k > 0 and (k & (k - 1)) == 0 else float(k) * self.dtu for k in ticks.flat])

    def _acc(self):
        return np.stack([self.out["ax"], self.out["ay"], self.out["az"]], 1)

    def _predicted(self):
        """v and u that every particle lends to the forces at time t."""
        dt = self.step_dt(self.t - self.t0)
        a = self._acc()
        v = self.vs + dt[:, None] * a
        u = self.us + dt * self.out["dudt"]
        return v, u

    def _evaluate(self, active: np.ndarray):
        """Lengths and densities of all, forces of the active particles."""
        if self.out is None:
            vel = (self.st["vx"], self.st["vy"], self.st["vz"])
            u = self.st["u"]
        else:
            v, u = self._predicted()
            vel = (v[:, 0], v[:, 1], v[:, 2])
        sinks = None if active.all() else np.nonzero(active)[0]
        o = O.compute_forces(self.st, self.prm, h_in=self.h, eps_in=self.eps, vel=vel, u=u, sinks=sinks,
                             alpha=self.st.get("alpha"), alpha_u=self.st.get("alpha_u"))
        if o["n_noconv"]:
            raise RuntimeError(f"{o['n_noconv']} length solves did not converge")
        if self.out is None:
            self.out = o
        else:
            for k, v in o.items():
                if k in _SINK_FIELDS:
                    self.out[k] = np.where(active, v, self.out[k])
                else:
                    self.out[k] = v
        self.h = self.out["h"].copy()
        self.eps = self.out["eps"].copy()
        self.sink_evals += int(active.sum())

    def _kick(self, idx: np.ndarray, dt: np.ndarray):
        """Half kick of the particles idx by dt/2 with their current rates."""
        st, o = self.st, self.out
        for c, ax in zip(("vx", "vy", "vz"), ("ax", "ay", "az")):
            st[c][idx] += 0.5 * dt * o[ax][idx]
        gas = idx[idx < self.n_gas]
        dg = dt[idx < self.n_gas]
        st["u"][gas] += 0.5 * dg * o["dudt"][gas]
        prm = self.prm
        if prm.alpha_switch:
            a = st["alpha"]
            a[gas] += 0.5 * dg * o["dalpha"][gas]
            a[gas] = np.where(a[gas] >= prm.alpha_min, a[gas], prm.alpha_min)
        if prm.conduction:
            a = st["alpha_u"]
            a[gas] += 0.5 * dg * o["dalpha_u"][gas]
            a[gas] = np.where(a[gas] >= prm.alpha_u_min, a[gas], prm.alpha_u_min)

    def criterion_ticks(self, idx: np.ndarray) -> np.ndarray:
        """Power-of-two step (ticks) of the criteria of Sect. 4.2, synchronised
        with the current tick."""
        dt = O.timestep_each(self.prm, self.st, self.out, self.eta_dt)[idx]
        lev = np.full(idx.size, self.L, np.int64)
        for k in range(idx.size):
            for n in range(self.L + 1):
                if math.ldexp(self.dt_max, -n) <= dt[k]:
                    lev[k] = n
                    break
        if self.common and idx.size:
            lev[:] = lev.max()
        ticks = np.left_shift(np.int64(1), self.L - lev)
        for k in range(idx.size):
            while self.t % ticks[k]:
                ticks[k] >>= 1
        return ticks

    def _start_steps(self, active: np.ndarray):
        """Criterion steps, wake-up, and the opening half kicks."""
        idx = np.nonzero(active)[0]
        c = self.criterion_ticks(idx)
        length = self.t1 - self.t0                     # ongoing steps of the others
        cur = length.copy()
        cur[idx] = c
        if self.wake and self.n_gas and self.prm.hydro and not self.common:
            gx = slice(0, self.n_gas)
            off, nb = O.neighbours(1, self.st["x"][gx], self.st["y"][gx], self.st["z"][gx], self.out["h"][gx],
                                   self.n_gas, period=self.prm.period)
            newlen = cur.copy()
            w = np.full(self.n, np.iinfo(np.int64).max)
            for i in range(self.n_gas):
                js = nb[off[i]:off[i + 1]]
                js = js[js != i]
                if js.size == 0:
                    continue
                if active[i]:
                    # at most f times the shortest step around it (a power of
                    # two below c_i divides c_i, hence the current tick)
                    cap = self.wake * int(cur[js].min())
                    newlen[i] = min(int(cur[i]), int(_pow2_floor(np.array([cap]))[0]))
                else:
                    act = js[active[js]]
                    if act.size:
                        w[i] = int(cur[act].min())
            # an inactive particle with a step longer than f w ends at t + w
            for j in range(self.n_gas):
                if active[j] or w[j] == np.iinfo(np.int64).max:
                    continue
                if length[j] > self.wake * w[j] and self.t + w[j] < self.t1[j]:
                    self._shorten(j, self.t + int(w[j]))
                    self.woken += 1
            self.last_c = cur
            c = newlen[idx]
        else:
            self.last_c = cur
        self.last_active = active.copy()
        self.t0[idx] = self.t
        self.t1[idx] = self.t + c
        self.vs[idx] = np.stack([self.st["vx"][idx], self.st["vy"][idx], self.st["vz"][idx]], 1)
        self.us[idx] = self.st["u"][idx]
        self._kick(idx, self.step_dt(c))

    def _shorten(self, j: int, end: int):
        """Wake particle j: its step now ends at tick ``end``; the opening half
        kick is redone from the synchronised state for the shorter step."""
        old = self.step_dt([self.t1[j] - self.t0[j]])[0]
        new = self.step_dt([end - self.t0[j]])[0]
        st, o = self.st, self.out
        for k, (c, ax) in enumerate(zip(("vx", "vy", "vz"), ("ax", "ay", "az"))):
            st[c][j] = self.vs[j, k] + 0.5 * new * o[ax][j]
        st["u"][j] = self.us[j] + 0.5 * new * o["dudt"][j]
        prm = self.prm
        if prm.alpha_switch:
            st["alpha"][j] = max(st["alpha"][j] - 0.5 * (old - new) * o["dalpha"][j], prm.alpha_min)
        if prm.conduction:
            st["alpha_u"][j] = max(st["alpha_u"][j] - 0.5 * (old - new) * o["dalpha_u"][j], prm.alpha_u_min)
        self.t1[j] = end

    def _drift(self, t_new: int):
        """Every particle to tick t_new with its half-kicked velocity (gas
        with the X-SPH correction), lengths along the drift as in Sect. 2.1."""
        d = self.step_dt([t_new - self.t])[0]
        st, o = self.st, self.out
        v = np.stack([st["vx"], st["vy"], st["vz"]], 1)
        if self.prm.xsph_eta > 0.0:
            v[:self.n_gas, 0] = v[:self.n_gas, 0] + o["xsph_x"][:self.n_gas]
            v[:self.n_gas, 1] = v[:self.n_gas, 1] + o["xsph_y"][:self.n_gas]
            v[:self.n_gas, 2] = v[:self.n_gas, 2] + o["xsph_z"][:self.n_gas]
        st["x"] += d * v[:, 0]
        st["y"] += d * v[:, 1]
        st["z"] += d * v[:, 2]
        L = self.prm.period
        if L > 0.0:  # back into the periodic box (Sect. 4.3)
            for k in ("x", "y", "z"):
                st[k] = st[k] - L * np.floor(st[k] / L)

        def factor(dv):
            f = 1.0 + (d / 3.0) * dv
            return np.where(f >= 0.5, np.where(f > 2.0, 2.0, f), 0.5)
        g = np.arange(self.n) < self.n_gas
        pos = g & (self.h > 0.0)
        self.h = np.where(pos, self.h * factor(o["divv"]), self.h)
        if self.prm.soft_mode != O.SOFT_CONSTANT:
            self.eps = np.where(self.eps > 0.0, self.eps * factor(o["divv_eps"]), self.eps)
        self.t = t_new

    # ---- one system time -------------------------------------------------
    def advance(self) -> np.ndarray:
        """Advance to the next step end; returns the active mask there."""
        t_new = int(self.t1.min())
        self._drift(t_new)
        active = self.t1 == self.t
        self._evaluate(active)
        idx = np.nonzero(active)[0]
        self._kick(idx, self.step_dt(self.t1[idx] - self.t0[idx]))
        if self.t == self.T:
            # every particle is synchronised at the end of the largest step
            self.t -= self.T
            self.t0 -= self.T
            self.t1 -= self.T
        self._start_steps(active)
        self.events += 1
        return active

    def run_to_sync(self) -> int:
        """Advance to the end of the current largest step (all synchronised)."""
        k = 0
        while True:
            self.advance()
            k += 1
            if self.t == 0:
                return k

    def synchronised_state(self) -> dict:
        """At a synchronisation point: the state with every particle's v, u at
        the current time (before its opening kick)."""
        assert np.all(self.t0 == self.t)
        s = dict(self.st)
        s["vx"], s["vy"], s["vz"] = self.vs[:, 0].copy(), self.vs[:, 1].copy(), self.vs[:, 2].copy()
        s["u"] = self.us.copy()
        return s
