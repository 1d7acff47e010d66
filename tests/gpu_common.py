"""Helpers shared by the GPU parity tests: run the HIP path through the C ABI
and the FP64 oracle on the same seeded inputs."""
import numpy as np

from paper_0912_1786_amd import tsph


def gpu_params(**kw):
    return tsph.tsph_default_params(**kw)


def oracle_params(orc, gp, walk_mode=None):
    """Oracle parameters equal to the GPU parameter block."""
    return orc.params(G=gp.G, theta=gp.theta, quadrupole=gp.quadrupole, soft_mode=gp.soft_mode,
                      eta_h=gp.eta_h, eta_eps=gp.eta_eps, gamma=gp.gamma, alpha=gp.alpha, beta=gp.beta,
                      av_eps2=gp.av_eps2, tc92=gp.tc92, h_maxit=gp.h_maxit, h_tol=gp.h_tol, kappa=gp.kappa,
                      leaf_size=gp.leaf_size, group_size=gp.group_size,
                      walk_mode=orc.WALK_GROUP if walk_mode is None else walk_mode,
                      nbr_mode=orc.NBR_TREE, gravity=gp.gravity, hydro=gp.hydro, batch_size=64,
                      batch_mode=0, grav_corr_literal=gp.grav_corr_literal, soften_cells=gp.soften_cells,
                      visc_form=gp.visc_form, entropy=gp.entropy, xsph_eta=gp.xsph_eta, h_scheme=gp.h_scheme,
                      h_weight=gp.h_weight, balsara=gp.balsara, alpha_switch=gp.alpha_switch,
                      alpha_min=gp.alpha_min, conduction=gp.conduction, alpha_u_min=gp.alpha_u_min,
                      period=gp.period)


def run_gpu(ic, gp, lists=0, eps_const=None):
    sim = tsph.Simulation(ic, gp, eps_const=eps_const)
    if lists:
        tsph.tsph_debug_lists(sim.ctx, lists)
    sim.compute_forces()
    flags, noconv = sim.flags()
    out = {k: sim.host(k) for k in ("ax", "ay", "az", "dudt", "rho", "pot", "h", "eps", "alpha", "alpha_u")}
    n = ic["n"]
    nf = len(tsph.SOLVE_FIELDS)
    solve = sim.export(tsph.DBG_SOLVE, np.float64, nf * n).reshape(nf, n)
    for i, name in enumerate(tsph.SOLVE_FIELDS):
        out[name] = solve[i]
    cnt = sim.export(tsph.DBG_COUNTS, np.int32, 3 * n).reshape(3, n)
    out["cnt_node"], out["cnt_pair"], out["cnt_sph"] = cnt
    if lists:
        out["lists"] = sim.export(tsph.DBG_NBR, np.int32, 3 * n * lists).reshape(3, n, lists)
    out["flags"], out["noconv"] = flags, noconv
    return sim, out


def acc(o):
    return np.stack([o["ax"], o["ay"], o["az"]], 1)


def relrms(a, b):
    den = np.sqrt(np.sum(b ** 2))
    return float(np.sqrt(np.sum((a - b) ** 2)) / den) if den > 0 else float(np.sqrt(np.sum((a - b) ** 2)))


def maxrel(a, b, mask=None):
    a, b = np.asarray(a), np.asarray(b)
    if mask is not None:
        a, b = a[mask], b[mask]
    if a.size == 0:
        return 0.0
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))
