#!/usr/bin/env python3
"""Throughput of the Tree+SPH step on one MI355X.

Workload: the two-species clustered field -- 1,048,576 gas + 1,048,576 dark
matter particles (DM:gas particle mass 5:1) in 64 Plummer halos inside a unit
cube, theta = 0.5 with quadrupoles, 60 neighbours for both h and eps,
adaptive softening with correction terms.  Inputs are seeded and synthetic
(paper_0912_1786_amd.inputs) and resident in HBM before timing.  Two
arithmetic forms are timed one after the other: the FP32-bulk form (gravity
interactions in single precision, the headline) and the plain FP64 form.

A step is one leapfrog step through the C ABI: kick-drift (half kick, drift,
predicted v and u), tsph_compute_forces (root cube, keys, radix sort, tree,
moments, h/eps solves and densities, gravity walk, SPH forces, output
scatter and time-step criteria) and the closing half kick.

Prints ONE JSON line: particle-steps/s = N * steps / wall time of the timed
steps, with a roofline entry for the dominant kernel (its duration measured
with HIP events recorded on its own stream inside the timed region) and the
FP64 oracle (built -O3 -march=native on this host) timed on the host's cores
for one step of the same workload.  "rows" adds the other configurations:
c1 (Evrard 4096, FP64: step and per-phase times, GPU and oracle), c2 (Evrard
262,144, 20 steps in both forms: step time, energy and momentum drift), c4
(256-member ensemble, one graph launch per step, autotuned leaf, group and
hand-off sizes), c5 (serving: closed-loop saturation, then p50/p99
latency under Poisson arrivals at 0.5x and 0.8x of it), f1 (individual
power-of-two time-steps on the 2M field: simulated time per wall second
against the global step) and options (the 2M field with each scheme option
alone: dissipation switches, periodic box, viscosity, entropy, X-SPH,
standard scheme, mass-density relation); "served_p50_ms" and
"served_p99_ms" are those at 0.5x.  --rows picks the rows to run.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (tree gravity+SPH) at N=2M, 1 GPU; served p50/p99 step latency"

# FP64 vector peak of MI355X: 256 CUs x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6
# FP32 vector peak of MI355X (published, with packed FP32 issue)
PEAK_FP32_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0

# Floating-point operations per interaction in the gravity walk kernel,
# counted from its source with FMA = 2, add/mul/div/sqrt/rsqrt = 1:
#   far node, monopole + quadrupole ........................... 49
#     (FP32-bulk form; the FP64 form's extra products by G are not counted)
#   near pair beyond 2 max(eps) (Newtonian branch) ............ 27
#   near pair inside 2 max(eps) (softened + correction terms) . 110
F_NODE, F_PAIR, F_SOFT = 49.0, 27.0, 110.0
# density solves, per candidate inside the kernel support at the converged
# length (one evaluation per solve and step is the least the method needs):
#   h solve over gas (W, dW/dh, rho, mass-weighted dW/dh, div v) ....... 45
#   eps solve over all species (W, dW/dh, mass-weighted d phi/d eps) ... 40
F_DENS_H, F_DENS_EPS = 45.0, 40.0
# SPH force pair (two kernel gradients, grad-h factors, pressure, AV) ..... 100
F_SPH = 100.0

# phase timed by the library -> kernel that dominates it and its source files
PHASE_KERNEL = {"density": ("k_density+k_density_sink", "density.hip"),
                "gravity": ("k_gravity+k_gravity_split+k_split_reduce", "gravity.hip"),
                "sph": ("k_sph+k_sph_split+k_sph_reduce", "sph.hip")}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_two_species_field_2M.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_id(src: str) -> str:
    """Hash of a kernel's source file and the shared header, without their
    // comments and blank lines: a traffic figure measured on other code is
    stale, one measured before a comment changed is not."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in (src, "tsph_internal.h"):
        with open(os.path.join(ROOT, "paper_0912_1786_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = re.sub(r"//.*$", "", line).rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, src: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the plain-copy calibration), or None
    when absent or taken on different source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    sid = kernel_source_id(src)
    for line in open(TRAFFIC_FILE):
        f = line.split()
        if len(f) >= 2 and f[0] == "kernel" and f[1] == kernel:
            kv = dict(x.split("=", 1) for x in f[2:] if "=" in x)
            if kv.get("source_id") == sid and "hbm_bytes_per_launch" in kv:
                return float(kv["hbm_bytes_per_launch"])
    return None


def algorithmic_flops(c: dict, phase: str, n: int, n_gas: int) -> float:
    if phase == "gravity":
        soft = c["softened_pairs_per_particle"]
        return n * (c["far_nodes_per_particle"] * F_NODE + (c["near_pairs_per_particle"] - soft) * F_PAIR
                    + soft * F_SOFT)
    if phase == "density":
        return (n_gas * c["density_h_candidates_per_gas_particle"] * F_DENS_H
                + n * c["density_eps_candidates_per_particle"] * F_DENS_EPS)
    return n_gas * c["sph_pairs_per_gas_particle"] * F_SPH


def copy_probe(mib: int):
    """A plain copy-like kernel of known size (float32 y = 1 * x over `mib`
    MiB, three launches): the calibration run for the HBM byte counters."""
    import torch
    n = mib * (1 << 20) // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n, "launches": 3}))


def run_form(args, ic, form: str, torch, tsph) -> dict:
    """Times args.steps KDK steps of one arithmetic form on resident inputs."""
    n = ic["n"]
    prec = tsph.FP32_BULK if form == "fp32_bulk" else tsph.FP64
    prm = tsph.tsph_default_params(nnei=60, theta=0.5, leaf_size=args.leaf, group_size=args.group,
                                   precision=prec)
    sim = tsph.Simulation(ic, prm, want_pot=False)
    log(f"[bench] {form}: N={n}; arena {tsph.tsph_bytes_required(n, prm) / 2**30:.2f} GiB")
    # first evaluation (cold start of h and eps) and the global time-step
    sim.compute_forces()
    dt = sim.timestep()
    flags, noconv = sim.flags()
    log(f"[bench] {form}: first force pass done: dt={dt:.3e} flags={flags:#x} noconv={noconv}")
    for w in range(args.warmup):
        sim.step(dt)
        torch.cuda.synchronize()
        log(f"[bench] {form}: warmup step {w + 1}/{args.warmup} done")
    tsph.tsph_timing(sim.ctx, True)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    t_wall0 = time.perf_counter()
    for k in range(args.steps):
        evs[k].record()
        sim.step(dt)
    evs[args.steps].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall0
    step_ms = [evs[k].elapsed_time(evs[k + 1]) for k in range(args.steps)]
    phases, calls = tsph.tsph_phase_times(sim.ctx)
    flags, noconv = sim.flags()
    sim.close()
    total_ms = sum(step_ms)
    log(f"[bench] {form}: timed {args.steps} steps: {total_ms:.1f} ms (wall {wall * 1e3:.1f} ms); per step "
        + ", ".join(f"{m:.1f}" for m in step_ms))
    log(f"[bench] {form}: phase ms/step: " + ", ".join(f"{k}={v / calls:.2f}" for k, v in phases.items()))
    # roofline of the dominant walk kernel
    dom = max(PHASE_KERNEL, key=lambda k: phases[k])
    kern, src = PHASE_KERNEL[dom]
    dom_ms = phases[dom] / calls
    roof = None
    cpath = os.path.join(ROOT, "oracle", "algorithmic_counts.json")
    if os.path.exists(cpath):
        c = json.load(open(cpath))
        if c["n"] == n and c["leaf_size"] == args.leaf:
            flops = algorithmic_flops(c, dom, n, ic["n_gas"])
            achieved = flops / (dom_ms / 1e3) / 1e12
            f32 = form == "fp32_bulk" and dom == "gravity"
            peak = PEAK_FP32_TFLOPS if f32 else PEAK_FP64_TFLOPS
            roof = {"kernel": kern, "bound": "alu", "achieved": round(achieved, 3), "peak": peak,
                    "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
                    "traffic": measured_traffic(f"{kern}/{form}", src), "algorithmic_flop_per_launch": flops,
                    "avg_launch_ms": round(dom_ms, 3), "arithmetic": "fp32" if f32 else "fp64",
                    "source_id": kernel_source_id(src)}
    return {"value": round(n * args.steps / (total_ms / 1e3), 1), "ms_per_step": round(total_ms / args.steps, 3),
            "median_step_ms": round(sorted(step_ms)[len(step_ms) // 2], 3),
            "phase_ms_per_step": {k: round(v / calls, 3) for k, v in phases.items()},
            "device_flags": flags, "roofline": roof}


def machine_probes(torch, tsph) -> dict:
    """Measured denominators on this GPU: the issue rate of independent FMA
    chains built as the walk kernels are (FP32 without packed issue, FP64)
    and the HBM bandwidth of a stream triad, each over three timed launches."""
    sink = torch.zeros(1, dtype=torch.float64, device="cuda")
    res = {}

    def timed(kind, n, *ptrs):
        tsph.tsph_probe(kind, n, *ptrs)  # warm-up
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        work = sum(tsph.tsph_probe(kind, n, *ptrs) for _ in range(3))
        e1.record()
        torch.cuda.synchronize()
        return work / (e0.elapsed_time(e1) / 1e3)

    res["fp32_fma_tflops"] = round(timed(tsph.PROBE_FMA32, 256, sink.data_ptr()) / 1e12, 2)
    res["fp64_fma_tflops"] = round(timed(tsph.PROBE_FMA64, 256, sink.data_ptr()) / 1e12, 2)
    n = 1 << 26
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b, c = torch.ones_like(a), torch.ones_like(a)
    res["hbm_triad_tbps"] = round(timed(tsph.PROBE_TRIAD, n, a.data_ptr(), b.data_ptr(), c.data_ptr()) / 1e12, 2)
    res["triad_bytes_per_launch"] = 24 * n
    del a, b, c
    return res


def load_native_oracle():
    """The FP64 oracle built -O3 -march=native for this host (into the
    ignored scratch folder gpurun_out/, or a temporary directory)."""
    import tempfile
    from oracle import build as obuild, oracle as O
    d = os.path.join(ROOT, "gpurun_out")
    try:
        os.makedirs(d, exist_ok=True)
    except OSError:
        d = tempfile.mkdtemp()
    path = obuild.build(out=os.path.join(d, "liboracle_native.so"), native=True)
    O.use_library(path)
    return O, "gcc -O3 -march=native -fopenmp -ffp-contract=off"


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            return next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        return ""


def oracle_step(O, ic, prm, dt: float = 1e-4):
    """One oracle step as the GPU runs it: force evaluation and the two half
    kicks.  Returns (wall seconds, per-phase seconds)."""
    t0 = time.perf_counter()
    out = O.compute_forces(ic, prm)
    st = {k: (v.copy() if hasattr(v, "copy") else v) for k, v in ic.items()}
    O.kick_drift(st, dt, 0, (out["ax"], out["ay"], out["az"]), out["dudt"])
    O.kick_drift(st, dt, 1, (out["ax"], out["ay"], out["az"]), out["dudt"])
    return time.perf_counter() - t0, out["t_phase"]


def cpu_baseline(O, build: str, nps: int, seed: int):
    """The FP64 oracle, as it stands, on the benchmark workload itself (the
    2M field by default): one full force evaluation plus the two half kicks."""
    from paper_0912_1786_amd import inputs
    ic = inputs.two_species_field(n_dm=nps, n_gas=nps, n_halo=64, seed=seed)
    prm = O.params(nnei=60, theta=0.5, leaf_size=16, group_size=64, walk_mode=O.WALK_GROUP)
    dt, ph = oracle_step(O, ic, prm)
    n = ic["n"]
    return {"value": n / dt, "unit": "particle-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(), "build": build,
            "phase_s": {k: round(v, 3) for k, v in ph.items()},
            "sample": f"one step of the benchmark recipe at N={n} (2x{nps}, seed {seed}): force evaluation "
                      f"(tree, h/eps solves, group walk, SPH) + KDK kicks, {dt:.2f} s wall"}


def row_c1(torch, tsph, O, steps: int = 20) -> dict:
    """Evrard sphere, 4096 gas particles, plain FP64: per-step time and the
    per-phase times of the GPU and of the oracle."""
    from paper_0912_1786_amd import inputs
    ic = inputs.evrard(4096, seed=1)
    prm = tsph.tsph_default_params(nnei=50, precision=tsph.FP64)
    sim = tsph.Simulation(ic, prm, want_pot=False)
    try:
        sim.compute_forces()
        dt = sim.timestep()
        for _ in range(3):
            sim.step(dt)
        tsph.tsph_timing(sim.ctx, True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(steps):
            sim.step(dt)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        phases, calls = tsph.tsph_phase_times(sim.ctx)
        flags, _ = sim.flags()
    finally:
        sim.close()
    od = O.params(nnei=50, theta=0.5, leaf_size=16, group_size=64, walk_mode=O.WALK_GROUP)
    wall, oph = oracle_step(O, ic, od)
    return {"workload": "evrard_4096_fp64", "n": 4096, "ms_per_step": round(ms, 3),
            "particle_steps_per_s": round(4096 / (ms / 1e3), 1),
            "phase_ms_per_step": {k: round(v / calls, 4) for k, v in phases.items()}, "device_flags": flags,
            "oracle_step_ms": round(wall * 1e3, 2), "oracle_phase_ms": {k: round(v * 1e3, 2) for k, v in oph.items()}}


def row_c2(n: int = 262144, steps: int = 20) -> dict:
    from paper_0912_1786_amd import runs
    out = {"workload": f"evrard_{n}_{steps}_steps"}
    for form in ("fp32_bulk", "fp64"):
        r = runs.evrard_run(n, steps, form)
        out[form] = {k: r[k] for k in ("median_step_ms", "particle_steps_per_s", "dE_over_E_step1",
                                         "dE_over_E_step20", "dP_rel_step1", "dP_rel_step20", "device_flags")}
    return out


def row_c4(members: int = 256, steps: int = 10) -> dict:
    from paper_0912_1786_amd import ensemble
    r = ensemble.run(members=members, steps=steps, warmup=2, tune=True, precision="fp32_bulk")
    return {k: r[k] for k in ("workload", "members", "n_total", "ms_per_step", "particle_steps_per_s",
                              "graph_launches_per_step", "leaf", "group", "split_leaves", "autotune_ms",
                              "device_flags")}


def row_c5(requests: int = 400) -> dict:
    from paper_0912_1786_amd import serve
    r = serve.run(n_sim=64, requests=requests)
    out = {k: r[k] for k in ("workload", "sims", "n_total", "streams", "hbm_budget_bytes", "evictions",
                             "admissions", "flagged")}
    out["saturation_requests_per_s"] = r["saturation"]["requests_per_s"]
    out["saturation_particle_steps_per_s"] = r["saturation"]["particle_steps_per_s"]
    for o in r["open_loop"]:
        tag = f"load_{o['rate_fraction']}"
        out[tag] = {k: o[k] for k in ("rate_per_s", "p50_ms", "p99_ms", "requests_per_s", "particle_steps_per_s")}
    return out


def row_f1(torch, tsph, nps: int = 1 << 20, events: int = 48, span: int = 64, seed: int = 1) -> dict:
    """Individual power-of-two time-steps on the 2M field (FP32 bulk): the
    largest step `span` times the global step of the first force pass, ten
    levels below it, wake-up factor 4.  Reports the simulated time advanced
    per wall second against the global-step loop at the global step."""
    from paper_0912_1786_amd import inputs
    ic = inputs.two_species_field(n_dm=nps, n_gas=nps, n_halo=64, seed=seed)
    prm = tsph.tsph_default_params(nnei=60, precision=tsph.FP32_BULK)
    sim = tsph.Simulation(ic, prm, want_pot=False)
    try:
        sim.compute_forces()
        dt = sim.timestep()
        for _ in range(2):
            sim.step(dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            sim.step(dt)
        torch.cuda.synchronize()
        global_ms = (time.perf_counter() - t0) * 1e3 / 3
    finally:
        sim.close()
    levels = 10
    sim = tsph.Simulation(ic, prm, want_pot=False)
    try:
        sim.block_start(span * dt, levels, 4)
        active = woken = 0
        ticks = prev = 0  # system time in ticks, counted across synchronisation points (t = 0)
        t0 = time.perf_counter()
        for _ in range(events):
            t, nact, nw = sim.block_advance()
            active += nact
            woken += nw
            ticks += (t - prev) if t > prev else (1 << levels) - prev + t
            prev = t
        wall_ms = (time.perf_counter() - t0) * 1e3
        flags, noconv = sim.flags()
    finally:
        sim.close()
    advanced = ticks * span / (1 << levels)  # in global steps
    return {"workload": "two_species_field_2M_individual_steps", "precision": "fp32_bulk", "largest_step_over_global": span,
            "levels": levels, "wake": 4, "events": events, "active_particle_steps": active, "woken": woken,
            "wall_ms": round(wall_ms, 1), "ms_per_event": round(wall_ms / events, 2),
            "advanced_in_global_steps": advanced, "ms_per_global_step_equivalent": round(wall_ms / advanced, 2),
            "global_step_ms": round(global_ms, 2), "speedup_in_simulated_time": round(global_ms * advanced / wall_ms, 2),
            "device_flags": flags, "noconv": noconv}


def row_options(torch, tsph, ic, steps: int = 5, warmup: int = 2) -> dict:
    """The 2M field (FP32 bulk) with each option of the scheme switched on
    alone, timed like the headline (KDK steps on resident inputs, HIP events)
    beside the plain form in the same row: the dissipation switches (f2), the
    periodic box with the Ewald correction on the field folded into the unit
    box (f3), and the scheme variants (f4)."""
    import numpy as np
    per = dict(ic)
    for k in ("x", "y", "z"):
        per[k] = np.mod(ic[k], 1.0)
    cases = {
        "plain": (ic, {}),
        "f2_switches": (ic, dict(balsara=1, alpha_switch=1, conduction=1)),
        "f3_periodic": (per, dict(period=1.0)),
        "f3_plain_folded": (per, {}),
        "f4_signal_viscosity": (ic, dict(visc_form=tsph.VISC_SIGNAL)),
        "f4_entropy": (ic, dict(entropy=1)),
        "f4_xsph": (ic, dict(xsph_eta=0.5)),
        "f4_standard_scheme": (ic, dict(h_scheme=tsph.H_STANDARD)),
        "f4_mass_density": (ic, dict(h_weight=tsph.HW_MASS)),
    }
    out = {"workload": "two_species_field_2M", "precision": "fp32_bulk", "steps": steps, "warmup": warmup}
    for name, (c, kw) in cases.items():
        prm = tsph.tsph_default_params(nnei=60, precision=tsph.FP32_BULK, **kw)
        sim = tsph.Simulation(c, prm, want_pot=False)
        try:
            sim.compute_forces()
            dt = sim.timestep()
            for _ in range(warmup):
                sim.step(dt)
            tsph.tsph_timing(sim.ctx, True)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(steps):
                sim.step(dt)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            phases, calls = tsph.tsph_phase_times(sim.ctx)
            flags, noconv = sim.flags()
        finally:
            sim.close()
        out[name] = {"ms_per_step": round(ms, 3), "particle_steps_per_s": round(c["n"] / (ms / 1e3), 1),
                     "phase_ms_per_step": {k: round(v / calls, 3) for k, v in phases.items()},
                     "device_flags": flags, "noconv": noconv}
        log(f"[bench] options: {name} {ms:.2f} ms/step")
    base = out["plain"]["ms_per_step"]
    for name in cases:
        out[name]["over_plain"] = round(out[name]["ms_per_step"] / base, 3)
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nps", type=int, default=1 << 20, help="particles per species")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--leaf", type=int, default=16)
    ap.add_argument("--group", type=int, default=64)
    ap.add_argument("--cpu-nps", type=int, default=1 << 20, help="per-species size of the oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true",
                    help="time only the 2M field (skip the Evrard, ensemble and serving configurations)")
    ap.add_argument("--rows", default="c1,c2,c4,c5,f1,options",
                    help="comma-separated rows to run besides the 2M field (c1, c2, c4, c5, f1, options)")
    ap.add_argument("--precision", choices=["both", "fp32_bulk", "fp64"], default="both",
                    help="arithmetic form(s) to time; with both, the FP32-bulk form is the headline")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run the copy kernel used to calibrate the HBM byte counters")
    args = ap.parse_args()
    want = set() if args.no_rows else {r.strip() for r in args.rows.split(",") if r.strip()}
    unknown = want - {"c1", "c2", "c4", "c5", "f1", "options"}
    if unknown:
        ap.error(f"unknown rows: {sorted(unknown)}")
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this engine has no multi-GPU path (each GPU would run its own "
              "simulations); run it with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_0912_1786_amd import inputs, tsph

    torch.cuda.set_device(0)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    t0 = time.time()
    ic = inputs.two_species_field(n_dm=args.nps, n_gas=args.nps, n_halo=64, seed=args.seed)
    n = ic["n"]
    log(f"[bench] N={n} inputs ready in {time.time() - t0:.1f}s")
    forms = {}
    for form in (["fp64", "fp32_bulk"] if args.precision == "both" else [args.precision]):
        forms[form] = run_form(args, ic, form, torch, tsph)
    head = forms["fp32_bulk"] if "fp32_bulk" in forms else forms["fp64"]
    headline = "fp32_bulk" if "fp32_bulk" in forms else "fp64"
    out = {
        "metric": METRIC, "value": head["value"], "unit": "particle-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if headline == "fp32_bulk" else "f64",
        "data": "synthetic",
        "config": {"workload": "two_species_field_2M", "n": n, "n_gas": ic["n_gas"], "n_dm": n - ic["n_gas"],
                   "halos": 64, "mass_ratio_dm_gas": 5, "theta": 0.5, "quadrupole": True, "nnei": 60,
                   "softening": "adaptive+corrections", "leaf_size": args.leaf, "group_size": args.group,
                   "precision": headline, "seed": args.seed},
        "phase_ms_per_step": head["phase_ms_per_step"],
        "median_step_ms": head["median_step_ms"],
        "device_flags": head["device_flags"],
        "roofline": head["roofline"],
    }
    for form, r in forms.items():
        if form != headline:
            out[f"{form}_form"] = r
    probe = machine_probes(torch, tsph)
    log(f"[bench] probes: {probe}")
    out["machine_probe"] = probe
    for r in [out["roofline"]] + [out[f"{f}_form"]["roofline"] for f in forms if f != headline]:
        if r:
            mp = probe["fp32_fma_tflops"] if r["arithmetic"] == "fp32" else probe["fp64_fma_tflops"]
            r["measured_peak"] = mp
            r["frac_of_measured_peak"] = round(r["achieved"] / mp, 4)
    O = obuild = None
    if not args.no_cpu_baseline or want:
        try:
            O, obuild = load_native_oracle()
        except Exception as e:  # no compiler on the host: the portable build
            log(f"[bench] native oracle build failed ({e}); using the portable -O2 build")
            from oracle import oracle as O
            obuild = "gcc -O2 -fopenmp -ffp-contract=off (native build failed)"
    if want:
        rows = {}
        for name, fn in (("c1", lambda: row_c1(torch, tsph, O)), ("c2", row_c2), ("c4", row_c4), ("c5", row_c5),
                         ("f1", lambda: row_f1(torch, tsph, nps=args.nps)),
                         ("options", lambda: row_options(torch, tsph, ic))):
            if name not in want:
                continue
            t1 = time.time()
            log(f"[bench] row {name} ...")
            try:
                rows[name] = fn()
            except Exception as e:  # a failing row is reported, not hidden, and does not drop the line
                rows[name] = {"error": f"{type(e).__name__}: {e}"}
            log(f"[bench] row {name} done in {time.time() - t1:.1f}s: {json.dumps(rows[name])[:300]}")
        out["rows"] = rows
        c5 = rows.get("c5", {})
        if "load_0.5" in c5:
            out["served_p50_ms"] = c5["load_0.5"]["p50_ms"]
            out["served_p99_ms"] = c5["load_0.5"]["p99_ms"]
    if not args.no_cpu_baseline:
        log("[bench] timing the oracle on the host ...")
        out["cpu_baseline"] = cpu_baseline(O, obuild, args.cpu_nps, args.seed)
        log(f"[bench] oracle: {out['cpu_baseline']['value']:.3e} particle-steps/s on "
            f"{out['cpu_baseline']['cores']} threads")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
