"""Serving resident simulations: single-step requests arrive for a
population of simulations; the server keeps particle and tree state on the
device, admits simulations within an HBM budget (least recently used idle
ones are moved to host memory when the budget is exceeded), and runs the
steps of different simulations concurrently on several streams
(continuous batching: a request is started as soon as a stream and its
simulation are free, while others are still running).

A step request runs one leapfrog step with the time-step taken on the
device (tsph_timestep, tsph_kick_drift_dt, tsph_compute_forces).  The step
of each resident simulation is captured once into a HIP graph when it is
admitted, so a request costs one graph launch on the host.  Requests of one
simulation run in arrival order; a simulation's result does not depend on
the mix it is served in.

    python -m paper_0912_1786_amd.serve --sims 64 --requests 400
"""
from __future__ import annotations

import argparse
import collections
import heapq
import json
import time

import numpy as np

from . import inputs, tsph

HOST_KEYS = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "vpx", "vpy", "vpz", "up", "h", "eps", "ax", "ay", "az",
             "dudt", "rho", "alpha", "alpha_u")


def population(n_sim: int = 64, seed: int = 2000, lo_log2: float = 12.0, hi_log2: float = 20.0):
    """Initial conditions: N = round(2^U(lo, hi)), gas fraction U(0, 1) (below
    64 gas particles the simulation is taken collisionless), Evrard sphere or
    Plummer sphere with equal probability, equal masses within a
    simulation.  Simulation k is drawn from seed + k."""
    out = []
    for k in range(n_sim):
        s = seed + k
        u = inputs.uniform(s, 900, 3)
        n = int(np.rint(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u[0])))
        n_gas = int(np.rint(u[1] * n))
        if n_gas < 64:
            n_gas = 0
        if u[2] < 0.5:
            ic = inputs.evrard(n, seed=s)
            ic["n_gas"] = n_gas
            ic["u"] = np.where(np.arange(n) < n_gas, ic["u"], 0.0)
            kind = "evrard"
        else:
            ic = inputs.plummer(n, seed=s, n_gas=n_gas, velocities=True)
            kind = "plummer"
        ic["kind"] = kind
        out.append(ic)
    return out


def capacity_class(n: int) -> int:
    """Shell capacity for a simulation of n particles: the next power of two
    (at least 2^12), so that simulations of similar size share shells."""
    return 1 << max(12, (int(n) - 1).bit_length())


class Shell:
    """A context and device buffers for up to `cap` particles, reused by the
    simulations admitted into it one after another (no allocation, no
    device-wide synchronisation on admission or eviction).  Keeps the
    captured step of each simulation that has run in it."""

    NAMES = tuple(k for k in tsph.Simulation.FIELDS if k != "pot")

    def __init__(self, cap: int, params):
        import torch
        self.cap = cap
        self.ctx = tsph.tsph_create(cap, params)
        dev = torch.device("cuda")
        self.bufs = {k: torch.zeros(cap, dtype=torch.float64, device=dev) for k in self.NAMES}
        self.bufs["dt"] = torch.zeros(1, dtype=torch.float64, device=dev)
        self.bufs["diag"] = torch.zeros(9, dtype=torch.float64, device=dev)
        self.graphs = {}  # simulation id -> its captured step in this shell
        self.last_use = 0.0

    @staticmethod
    def bytes_for(cap: int, params) -> int:
        return tsph.tsph_bytes_required(cap, params) + 8 * (len(Shell.NAMES) * cap + 10)

    def close(self):
        self.graphs.clear()
        if self.ctx is not None:
            tsph.tsph_destroy(self.ctx)
            self.ctx = None
        self.bufs = None


class Resident:
    """One simulation: its initial conditions, and while admitted the shell
    holding its device state."""

    def __init__(self, sid: int, ic: dict, params):
        self.sid, self.ic, self.params = sid, ic, params
        self.sim = None          # tsph.Simulation in a shell while resident
        self.shell = None
        self.graph = None        # its captured step while resident
        self.saved = None        # pinned host copy of the state while evicted
        self.busy = False
        self.steps = 0
        self.last_use = 0.0
        self.flag_bits = 0       # device flags raised while it was resident in earlier shells
        self.noconv = 0
        self.flag_words = []     # pinned (flags, unconverged) taken at evictions, not read yet

    @property
    def n(self) -> int:
        return int(self.ic["n"])

    def bytes(self) -> int:
        return Shell.bytes_for(capacity_class(self.n), self.params)

    def admit(self, shell: Shell, capture_stream=None):
        import torch
        if self.sim is not None:
            return
        if self.saved is None:
            self.sim = tsph.Simulation(self.ic, self.params, want_pot=False, ctx=shell.ctx, bufs=shell.bufs)
            self.sim.compute_forces()  # cold start: lengths and forces of the initial state
        else:
            # the state and the context's carry to the next step: the
            # simulation continues exactly where it left the device.  The
            # copies come from pinned memory without waiting: they are
            # ordered on the current stream after the eviction's copies out,
            # and the step's stream waits for the current stream.
            src = dict(self.saved, n=self.n, n_gas=int(self.ic["n_gas"]))
            self.sim = tsph.Simulation(src, self.params, want_pot=False, ctx=shell.ctx, bufs=shell.bufs, fill=False)
            for k in HOST_KEYS:
                self.sim.a[k].copy_(self.saved[k], non_blocking=True)
            carry = self.saved["carry"].to(self.sim.a["x"].device, non_blocking=True)
            tsph.tsph_carry_load(shell.ctx, self.n, carry.data_ptr())
        self.shell = shell
        g = shell.graphs.get(self.sid) if capture_stream is not None else None
        if g is None and capture_stream is not None:
            capture_stream.wait_stream(torch.cuda.current_stream())
            g = torch.cuda.CUDAGraph()
            with torch.cuda.stream(capture_stream):
                g.capture_begin()
                self.sim.device_step(capture_stream)
                g.capture_end()
            shell.graphs[self.sid] = g
        self.graph = g

    def launch(self, stream):
        """Issues one step on `stream`: the captured graph, or the calls."""
        import torch
        if self.graph is not None:
            with torch.cuda.stream(stream):
                self.graph.replay()
        else:
            self.sim.device_step(stream)

    def evict(self) -> Shell:
        """Moves the state, the carry and the device flags to pinned host
        memory (copies ordered on the current stream, not waited for: the
        simulation is idle, its last step complete) and hands back the
        shell, whose flags start clean for the next occupant."""
        import torch
        if self.saved is None:
            self.saved = {k: torch.empty(self.n, dtype=torch.float64, pin_memory=True) for k in HOST_KEYS}
            self.saved["carry"] = torch.empty(tsph.tsph_carry_bytes(self.n) // 8, dtype=torch.float64,
                                              pin_memory=True)
        for k in HOST_KEYS:
            self.saved[k].copy_(self.sim.a[k], non_blocking=True)
        carry = torch.empty(self.saved["carry"].numel(), dtype=torch.float64, device=self.sim.a["x"].device)
        tsph.tsph_carry_save(self.sim.ctx, self.n, carry.data_ptr())
        self.saved["carry"].copy_(carry, non_blocking=True)
        words = torch.zeros(2, dtype=torch.int32, pin_memory=True)
        tsph.tsph_take_flags_async(self.sim.ctx, words.data_ptr())
        self.flag_words.append(words)
        shell = self.shell
        self.sim.close()  # borrowed context: left as it is
        self.sim, self.shell, self.graph = None, None, None
        return shell

    def harvest_flags(self):
        """Adds the flags taken at evictions to its own (after the device
        has passed those copies)."""
        for w in self.flag_words:
            self.flag_bits |= int(w[0]) & 0xffffffff
            self.noconv += int(w[1])
        self.flag_words = []

    def host(self, k):
        """Host copy of array k of the state, resident or not."""
        if self.sim is not None:
            return self.sim.host(k)
        import torch
        torch.cuda.synchronize()  # the eviction's copies out are not waited for
        return self.saved[k].numpy().copy()


class Server:
    def __init__(self, ics, streams: int = 8, hbm_budget: int | None = None, precision: int = tsph.FP32_BULK,
                 graphs: bool = True):
        import torch
        self.torch = torch
        self.res = []
        self.params = tsph.tsph_default_params(nnei=50.0, precision=precision)
        for k, ic in enumerate(ics):
            self.res.append(Resident(k, ic, self.params))
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        self.capture_stream = torch.cuda.Stream() if graphs else None
        self.free = list(range(len(self.streams)))
        self.budget = hbm_budget
        self.pool = []            # shells not holding a simulation
        self.shell_bytes = 0      # all shells, in use or pooled
        self.evictions = 0
        self.admissions = 0
        self.shells_made = 0

    def _drop_pooled(self) -> bool:
        """Destroys the least recently used pooled shell."""
        if not self.pool:
            return False
        sh = min(self.pool, key=lambda x: x.last_use)
        self.pool.remove(sh)
        self.shell_bytes -= Shell.bytes_for(sh.cap, self.params)
        sh.close()
        return True

    def _ensure_resident(self, r: Resident, now: float) -> bool:
        """Admits r if needed; False when the budget cannot make room now."""
        if r.sim is not None:
            return True
        cap = capacity_class(r.n)
        shell = next((x for x in self.pool if x.cap == cap), None)
        if shell is None:
            need = Shell.bytes_for(cap, self.params)
            if self.budget is not None:
                # an idle simulation of the same capacity class gives up its
                # shell directly (no context destroyed and made again)
                same = [x for x in self.res if x.sim is not None and not x.busy and x.shell.cap == cap]
                if same and self.shell_bytes + need > self.budget:
                    v = min(same, key=lambda x: x.last_use)
                    shell = v.evict()
                    shell.last_use = now
                    self.evictions += 1
                while shell is None and self.shell_bytes + need > self.budget:
                    if self._drop_pooled():
                        continue
                    idle = [x for x in self.res if x.sim is not None and not x.busy]
                    if not idle:
                        break
                    v = min(idle, key=lambda x: x.last_use)
                    sh = v.evict()
                    sh.last_use = now
                    self.evictions += 1
                    if sh.cap == cap:
                        shell = sh
                        break
                    self.pool.append(sh)
                if shell is None and self.shell_bytes + need > self.budget and any(
                        x.sim is not None for x in self.res):
                    return False
            if shell is None:
                shell = Shell(cap, self.params)
                self.shell_bytes += need
                self.shells_made += 1
        else:
            self.pool.remove(shell)
        r.admit(shell, self.capture_stream)
        self.admissions += 1
        return True

    def run(self, arrivals, closed_loop: bool = False, duration: float | None = None, seed: int = 1,
            max_seconds: float = 120.0):
        """Serves requests.  arrivals: list of (time_s, sim id), times relative
        to the start (open loop).  closed_loop: every free stream is given a
        request for a random idle simulation at once, for `duration` seconds.
        Returns the per-request records; raises after max_seconds."""
        torch = self.torch
        rng = np.random.default_rng(seed)
        pending = collections.deque(sorted(arrivals))
        waiting = []       # (arrival, seq, sid) ready but not started
        inflight = []      # (event, slot, resident, arrival, start)
        done = []
        seq = 0
        t0 = time.perf_counter()
        while True:
            now = time.perf_counter() - t0
            if now > max_seconds:
                raise RuntimeError(f"serving loop still busy after {max_seconds} s: {len(waiting)} waiting, "
                                   f"{len(inflight)} in flight, {len(pending)} not arrived")
            while pending and pending[0][0] <= now:
                a, sid = pending.popleft()
                heapq.heappush(waiting, (a, seq, sid))
                seq += 1
            if closed_loop:
                if now < duration:
                    idle = [x.sid for x in self.res if not x.busy and x.sid not in {w[2] for w in waiting}]
                    while len(waiting) < len(self.free) and idle:
                        sid = idle.pop(int(rng.integers(len(idle))))
                        heapq.heappush(waiting, (now, seq, sid))
                        seq += 1
                elif not inflight and not waiting:
                    break
            elif not pending and not waiting and not inflight:
                break
            # completions
            still = []
            for ev, slot, r, a, st in inflight:
                if ev.query():
                    t = time.perf_counter() - t0
                    r.busy = False
                    r.steps += 1
                    r.last_use = t
                    self.free.append(slot)
                    done.append({"sim": r.sid, "n": r.n, "arrival": a, "start": st, "end": t})
                else:
                    still.append((ev, slot, r, a, st))
            inflight = still
            # starts: oldest waiting request whose simulation is free
            deferred = []
            while self.free and waiting:
                a, s, sid = heapq.heappop(waiting)
                r = self.res[sid]
                if r.busy:
                    deferred.append((a, s, sid))
                    continue
                if not self._ensure_resident(r, now):
                    deferred.append((a, s, sid))
                    break
                slot = self.free.pop()
                stream = self.streams[slot]
                r.busy = True
                st = time.perf_counter() - t0
                stream.wait_stream(torch.cuda.current_stream())  # the admission's own work
                r.launch(stream)
                ev = torch.cuda.Event()
                ev.record(stream)
                inflight.append((ev, slot, r, a, st))
            for d in deferred:
                heapq.heappush(waiting, d)
            if not inflight and not self.free:
                raise RuntimeError("no stream free and nothing in flight")
            time.sleep(0.0002)
        torch.cuda.synchronize()
        return done

    def flags(self):
        """(sid, (flag bits, unconverged solves)) of every simulation since
        the previous call: what its shells raised while it was resident,
        including earlier residencies."""
        self.torch.cuda.synchronize()  # the evictions' flag copies are done
        out = []
        for r in self.res:
            r.harvest_flags()
            f, nc = r.sim.flags() if r.sim is not None else (0, 0)
            out.append((r.sid, (r.flag_bits | f, r.noconv + nc)))
            r.flag_bits, r.noconv = 0, 0
        return out

    def close(self):
        self.torch.cuda.synchronize()
        for r in self.res:
            if r.sim is not None:
                r.sim.close()
                self.pool.append(r.shell)
                r.sim, r.shell, r.graph = None, None, None
        while self._drop_pooled():
            pass


def poisson_arrivals(rate: float, count: int, n_sim: int, seed: int = 3):
    """Open-loop arrivals: exponential gaps at `rate` per second, each naming a
    uniformly random simulation."""
    gaps = -np.log(inputs.uniform_open(seed, 950, count)) / rate
    t = np.cumsum(gaps)
    sims = np.minimum((inputs.uniform(seed, 951, count) * n_sim).astype(np.int64), n_sim - 1)
    return [(float(a), int(s)) for a, s in zip(t, sims)]


def summarize(done, label: str) -> dict:
    lat = np.array([d["end"] - d["arrival"] for d in done]) * 1e3
    span = max(d["end"] for d in done) - min(d["arrival"] for d in done)
    ps = sum(d["n"] for d in done)
    return {"label": label, "requests": len(done), "p50_ms": round(float(np.percentile(lat, 50)), 3),
            "p99_ms": round(float(np.percentile(lat, 99)), 3), "requests_per_s": round(len(done) / span, 2),
            "particle_steps_per_s": round(ps / span, 1)}


def run(n_sim: int = 64, requests: int = 400, streams: int = 8, budget_fraction: float = 0.5, seed: int = 2000,
        saturation_s: float = 3.0, warmup_s: float = 2.0) -> dict:
    """Closed-loop saturation throughput (after a closed-loop warm-up that
    admits the first simulations and takes their cold starts), then
    open-loop Poisson arrivals at 0.5x and 0.8x of it; the HBM budget is
    budget_fraction of what the whole population would hold."""
    import torch
    ics = population(n_sim, seed)
    probe = Server(ics, streams)
    total = sum(r.bytes() for r in probe.res)
    budget = int(budget_fraction * total)
    probe.close()
    srv = Server(ics, streams, hbm_budget=budget)
    try:
        if warmup_s > 0:
            srv.run([], closed_loop=True, duration=warmup_s, seed=seed + 7)
        sat = srv.run([], closed_loop=True, duration=saturation_s)
        s0 = summarize(sat, "closed_loop_saturation")
        out = {"workload": f"serving_{n_sim}_sims", "sims": n_sim, "n_total": int(sum(ic["n"] for ic in ics)),
               "streams": streams, "hbm_budget_bytes": budget, "population_bytes": total,
               "saturation": s0, "open_loop": []}
        for frac in (0.5, 0.8):
            rate = frac * s0["requests_per_s"]
            arr = poisson_arrivals(rate, requests, n_sim, seed=int(seed + 100 * frac))
            done = srv.run(arr)
            out["open_loop"].append({"rate_fraction": frac, "rate_per_s": round(rate, 2), **summarize(done, f"{frac}x")})
        out["evictions"] = srv.evictions
        out["admissions"] = srv.admissions
        out["flagged"] = [(sid, f) for sid, f in srv.flags() if f != (0, 0)][:8]
        torch.cuda.synchronize()
        return out
    finally:
        srv.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--sims", type=int, default=64)
    ap.add_argument("--requests", type=int, default=400)
    ap.add_argument("--streams", type=int, default=8)
    ap.add_argument("--budget-fraction", type=float, default=0.5)
    ap.add_argument("--seed", type=int, default=2000)
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(run(a.sims, a.requests, a.streams, a.budget_fraction, a.seed)), flush=True)


if __name__ == "__main__":
    main()
