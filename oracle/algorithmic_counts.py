"""Per-particle interaction counts of the method on the 2M two-species field
(test/benchmark infrastructure; calls only the oracle).

The counts are what the method itself must evaluate per particle and step:
the oracle's per-particle Barnes-Hut walk (Sect. 2.2, theta = 0.5 with
quadrupoles, Dubinski opening test plus the softening-clear rule) gives the
far-node and near-pair interactions, and its neighbour definitions give the
SPH pairs (r < 2 max(h_i, h_j), Sect. 3.1) and density candidates (r < 2 h_i
for gas, r < 2 eps_i for all).  The GPU's grouped walk evaluates more than
these; only these count as algorithmic work.

Writes oracle/algorithmic_counts.json.  Usage:
    python oracle/algorithmic_counts.py [--sample 4096] [--nps 1048576]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
from paper_0912_1786_amd import inputs  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nps", type=int, default=1 << 20, help="particles per species")
    ap.add_argument("--sample", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--leaf", type=int, default=16)
    a = ap.parse_args()
    t0 = time.time()
    ic = inputs.two_species_field(n_dm=a.nps, n_gas=a.nps, n_halo=64, seed=a.seed)
    n = ic["n"]
    rng = np.random.default_rng(12345)
    sinks = np.sort(rng.choice(n, a.sample, replace=False))
    prm = O.params(nnei=60, theta=0.5, leaf_size=a.leaf, group_size=64, walk_mode=O.WALK_PARTICLE)
    o = O.compute_forces(ic, prm, sinks=sinks)
    x, y, z = ic["x"], ic["y"], ic["z"]
    gas = sinks[sinks < ic["n_gas"]]
    # density candidates inside the kernel support (gas: h over gas; all: eps over all)
    pos = np.stack([x, y, z], 1)
    gpos = pos[: ic["n_gas"]]
    dens_h, eps_cnt = [], []
    for s in sinks:
        d2 = np.sum((pos - pos[s]) ** 2, 1)
        eps_cnt.append(int(np.count_nonzero(d2 < (2.0 * o["eps"][s]) ** 2)))
        if s < ic["n_gas"]:
            dens_h.append(int(np.count_nonzero(d2[: ic["n_gas"]] < (2.0 * o["h"][s]) ** 2)))
    dens_h = np.array(dens_h)
    del gpos
    out = {
        "workload": "two_species_field", "n": int(n), "n_gas": int(ic["n_gas"]), "seed": a.seed,
        "theta": 0.5, "nnei": 60, "leaf_size": a.leaf, "sample_sinks": int(a.sample),
        "far_nodes_per_particle": float(o["cnt_node"][sinks].mean()),
        "near_pairs_per_particle": float(o["cnt_pair"][sinks].mean()),
        "softened_pairs_per_particle": float(o["cnt_soft"][sinks].mean()),
        "sph_pairs_per_gas_particle": float(o["cnt_sph"][gas].mean()),
        "density_h_candidates_per_gas_particle": float(dens_h.mean()),
        "density_eps_candidates_per_particle": float(np.mean(eps_cnt)),
        "newton_passes_per_particle_cold": float(o["iters"].mean()),
        "oracle_seconds": round(time.time() - t0, 1),
        "oracle_threads": O.num_threads(),
    }
    path = os.path.join(HERE, "algorithmic_counts.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
