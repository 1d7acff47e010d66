"""Ensembles of independent simulations advanced by one HIP-graph launch per
step, with the leaf and group sizes and the hand-off share chosen by a measuring
autotuner.

The members live in one context as a forest (tsph_set_members): their
particles are held back to back, every tree-build stage and every walk is
one launch over all members (a sort segmented by member, one root per
member, walk batches of all members in one work queue), and each member
keeps its own time-step.  The step of all members -- time-step criteria,
kick-drift, force evaluation and the closing kick, with each member's
time-step read on the device -- is captured once into a HIP graph and
replayed with a single launch per step.  Members share no data, so each
member's result does not depend on the others: the tests require the
ensemble step to equal the member stepped alone in a context of its own,
bit for bit.

    python -m paper_0912_1786_amd.ensemble --members 256 --steps 10
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

from . import inputs, tsph

# (leaf size, walk-group size, split_leaves) tried by the autotuner: the tree
# leaves, the sinks sharing a walk, and how much of a batch's near field or
# candidate set its own wavefront evaluates before handing the rest on
CANDIDATES = ((8, 32, 256), (16, 32, 256), (16, 64, 256), (32, 64, 256), (16, 64, 128), (16, 64, 512))


def ensemble_ics(members: int, seed: int = 1000):
    """Evrard spheres with N log-uniform in [2^10, 2^15] and u0 uniform in
    [0.02, 0.1]; member k is drawn from seed + k."""
    sizes, u0 = inputs.ensemble_sizes(members, seed)
    return [inputs.evrard(int(n), seed=seed + k, u0=float(u)) for k, (n, u) in enumerate(zip(sizes, u0))]


def member_params(nnei: float = 50.0, precision: int = tsph.FP32_BULK, leaf: int = 16, group: int = 64,
                  split: int = 256):
    return tsph.tsph_default_params(nnei=nnei, leaf_size=leaf, group_size=group, precision=precision,
                                    split_leaves=split)


def autotune(ics, nnei: float = 50.0, precision: int = tsph.FP32_BULK, reps: int = 3) -> dict:
    """Times warm force evaluations of the whole ensemble (one context
    holding every member) under each candidate (leaf, group, split_leaves)
    and keeps the fastest.  Returns {"leaf", "group", "split", "ms":
    {candidate: ms}}."""
    import torch
    big, members = tsph.concat_ics(ics)
    times = {}
    for cand in CANDIDATES:
        leaf, group, split = cand
        sim = tsph.Simulation(big, member_params(nnei, precision, leaf, group, split), want_pot=False,
                              members=members)
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
            times[cand] = a.elapsed_time(b) / reps
        finally:
            sim.close()
    best = min(times, key=times.get)
    return {"leaf": best[0], "group": best[1], "split": best[2], "ms": times}


class Ensemble:
    """Independent simulations in one context, stepped by one graph launch."""

    def __init__(self, ics, nnei: float = 50.0, precision: int = tsph.FP32_BULK, leaf: int = 16, group: int = 64,
                 split: int = 256):
        import torch
        self.torch = torch
        big, members = tsph.concat_ics(ics)
        self.params = member_params(nnei, precision, leaf, group, split)
        self.sim = tsph.Simulation(big, self.params, want_pot=False, members=members)
        self.count = len(ics)
        self.n_total = self.sim.n
        self.graph = None
        self.stream = torch.cuda.Stream()

    def first_forces(self):
        """Cold-start force evaluation of every member (outside any graph)."""
        self.sim.compute_forces()
        self.torch.cuda.synchronize()

    def eager_step(self):
        """One step of every member, issued call by call on the current
        stream (what the graph replays)."""
        self.sim.device_step()

    def capture(self):
        """Captures one step of all members into a graph."""
        torch = self.torch
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            self.sim.device_step(self.stream)
        torch.cuda.synchronize()
        self.graph = g
        return g

    def step(self):
        self.graph.replay()

    def member(self, k: int, key: str):
        return self.sim.member(k, key)

    def flags(self):
        return self.sim.flags()

    def close(self):
        self.graph = None
        if self.sim is not None:
            self.sim.close()
            self.sim = None


def run(members: int = 256, steps: int = 10, warmup: int = 2, seed: int = 1000, tune: bool = True,
        precision: str = "fp32_bulk") -> dict:
    import torch
    t0 = time.time()
    ics = ensemble_ics(members, seed)
    prec = tsph.FP32_BULK if precision == "fp32_bulk" else tsph.FP64
    tuning = autotune(ics, precision=prec) if tune else None
    t_tune = time.time() - t0
    leaf, group, split = (tuning["leaf"], tuning["group"], tuning["split"]) if tuning else (16, 64, 256)
    ens = Ensemble(ics, precision=prec, leaf=leaf, group=group, split=split)
    try:
        ens.first_forces()
        ens.capture()
        for _ in range(warmup):
            ens.step()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        # replays are launched on the current stream
        a.record()
        for _ in range(steps):
            ens.step()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / steps
        flags, noconv = ens.flags()
        return {"workload": f"evrard_ensemble_{members}", "members": members, "n_total": ens.n_total,
                "precision": precision, "steps": steps, "ms_per_step": round(ms, 3),
                "particle_steps_per_s": round(ens.n_total / (ms / 1e3), 1), "graph_launches_per_step": 1,
                "leaf": leaf, "group": group, "split_leaves": split,
                "autotune_ms": None if tuning is None else
                {f"{l}x{g}x{sp}": round(t, 3) for (l, g, sp), t in tuning["ms"].items()},
                "autotune_s": round(t_tune, 1), "device_flags": flags, "noconv": noconv}
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
