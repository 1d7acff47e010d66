"""Ensembles of independent simulations advanced by one HIP-graph launch per
step, with the leaf and group sizes chosen by a measuring autotuner.

Every member keeps its own context, device state and time-step.  The step
of all members -- time-step criteria, kick-drift, force evaluation and the
closing kick, with the time-step read on the device -- is captured once
into a HIP graph across several streams (members spread over them) and
replayed with a single launch per step.  Members share no data, so each
member's result does not depend on the others: the tests require the
ensemble step to equal the member stepped alone, bit for bit.

    python -m paper_0912_1786_amd.ensemble --members 256 --steps 10
"""
from __future__ import annotations

import argparse
import json
import math
import time

import numpy as np

from . import inputs, tsph

# leaf and group sizes tried by the autotuner
CANDIDATES = ((8, 32), (16, 32), (16, 64), (32, 64))


def ensemble_ics(members: int, seed: int = 1000):
    """Evrard spheres with N log-uniform in [2^10, 2^15] and u0 uniform in
    [0.02, 0.1]; member k is drawn from seed + k."""
    sizes, u0 = inputs.ensemble_sizes(members, seed)
    return [inputs.evrard(int(n), seed=seed + k, u0=float(u)) for k, (n, u) in enumerate(zip(sizes, u0))]


def size_class(n: int) -> int:
    """Autotuner classes: one per factor of two in N."""
    return int(math.floor(math.log2(max(n, 1))))


def autotune(ics, nnei: float = 50.0, precision: int = tsph.FP32_BULK, reps: int = 3) -> dict:
    """For each size class of the ensemble, times one warm force evaluation
    of its largest member under every candidate (leaf, group) and keeps the
    fastest.  Returns {class: (leaf, group, {candidate: ms})}."""
    import torch
    by_class = {}
    for ic in ics:
        c = size_class(ic["n"])
        if c not in by_class or ic["n"] > by_class[c]["n"]:
            by_class[c] = ic
    choice = {}
    for c, ic in sorted(by_class.items()):
        times = {}
        for leaf, group in CANDIDATES:
            prm = tsph.tsph_default_params(nnei=nnei, leaf_size=leaf, group_size=group, precision=precision)
            sim = tsph.Simulation(ic, prm, want_pot=False)
            try:
                sim.compute_forces()
                torch.cuda.synchronize()
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record()
                for _ in range(reps):
                    sim.compute_forces()
                b.record()
                torch.cuda.synchronize()
                times[(leaf, group)] = a.elapsed_time(b) / reps
            finally:
                sim.close()
        best = min(times, key=times.get)
        choice[c] = (best[0], best[1], times)
    return choice


class Ensemble:
    """Independent simulations stepped together by one graph launch."""

    def __init__(self, ics, nnei: float = 50.0, precision: int = tsph.FP32_BULK, tuning: dict | None = None,
                 streams: int = 16):
        import torch
        self.torch = torch
        self.members = []
        self.params = []
        for ic in ics:
            leaf, group = (16, 64)
            if tuning is not None:
                leaf, group = tuning[size_class(ic["n"])][:2]
            prm = tsph.tsph_default_params(nnei=nnei, leaf_size=leaf, group_size=group, precision=precision)
            self.params.append(prm)
            self.members.append(tsph.Simulation(ic, prm, want_pot=False))
        self.n_total = sum(m.n for m in self.members)
        self.streams = [torch.cuda.Stream() for _ in range(max(1, streams))]
        self.graph = None

    def first_forces(self):
        """Cold-start force evaluation of every member (outside any graph)."""
        for m in self.members:
            m.compute_forces()
        self.torch.cuda.synchronize()

    def eager_step(self):
        """One step of every member, issued member by member on the current
        stream (the reference the graph is checked against)."""
        for m in self.members:
            m.device_step()

    def capture(self):
        """Captures one step of all members into a graph; members are spread
        over the streams, which fork from and join the capture stream."""
        torch = self.torch
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        main = torch.cuda.Stream()
        with torch.cuda.graph(g, stream=main):
            for s in self.streams:
                s.wait_stream(main)
            for k, m in enumerate(self.members):
                m.device_step(self.streams[k % len(self.streams)])
            for s in self.streams:
                main.wait_stream(s)
        torch.cuda.synchronize()
        self.graph = g
        return g

    def step(self):
        self.graph.replay()

    def flags(self):
        out = []
        for m in self.members:
            out.append(m.flags())
        return out

    def close(self):
        for m in self.members:
            m.close()
        self.members = []
        self.graph = None


def run(members: int = 256, steps: int = 10, warmup: int = 2, seed: int = 1000, tune: bool = True,
        precision: str = "fp32_bulk") -> dict:
    import torch
    t0 = time.time()
    ics = ensemble_ics(members, seed)
    prec = tsph.FP32_BULK if precision == "fp32_bulk" else tsph.FP64
    tuning = autotune(ics, precision=prec) if tune else None
    t_tune = time.time() - t0
    ens = Ensemble(ics, precision=prec, tuning=tuning)
    try:
        ens.first_forces()
        ens.capture()
        for _ in range(warmup):
            ens.step()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(steps):
            ens.step()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        bad = [(i, f) for i, f in enumerate(ens.flags()) if f != (0, 0)]
        return {"workload": f"evrard_ensemble_{members}", "members": members, "n_total": ens.n_total,
                "precision": precision, "steps": steps, "ms_per_step": round(ms, 3),
                "particle_steps_per_s": round(ens.n_total / (ms / 1e3), 1), "graph_launches_per_step": 1,
                "autotune": None if tuning is None else
                {str(c): {"leaf": v[0], "group": v[1], "ms": {f"{l}x{g}": round(t, 3) for (l, g), t in v[2].items()}}
                 for c, v in tuning.items()},
                "autotune_s": round(t_tune, 1), "members_flagged": bad[:8]}
    finally:
        ens.close()


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--members", type=int, default=256)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--precision", choices=["fp32_bulk", "fp64"], default="fp32_bulk")
    a = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(run(a.members, a.steps, a.warmup, a.seed, not a.no_tune, a.precision)), flush=True)


if __name__ == "__main__":
    main()
