"""ctypes binding of the FP64 CPU oracle (TEST INFRASTRUCTURE ONLY).

Only the test-suite, the smoke check and the benchmark's CPU-baseline leg use
this module.  It never imports the HIP package and the HIP package never
imports it.  All arrays are float64 numpy arrays in caller order (gas first).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

D = C.POINTER(C.c_double)
I64 = C.POINTER(C.c_int64)
I32 = C.POINTER(C.c_int32)
U64 = C.POINTER(C.c_uint64)

SOFT_ADAPTIVE, SOFT_CONSTANT, SOFT_ADAPTIVE_NOCORR = 0, 1, 2
WALK_PARTICLE, WALK_GROUP, WALK_DIRECT = 0, 1, 2
NBR_TREE, NBR_BRUTE = 0, 1
VISC_MG, VISC_SIGNAL = 0, 1
H_LAGRANGIAN, H_STANDARD = 0, 1
HW_NUMBER, HW_MASS = 0, 1


class Params(C.Structure):
    _fields_ = [("G", C.c_double), ("theta", C.c_double), ("quadrupole", C.c_int32),
                ("soft_mode", C.c_int32), ("eta_h", C.c_double), ("eta_eps", C.c_double),
                ("gamma", C.c_double), ("alpha", C.c_double), ("beta", C.c_double),
                ("av_eps2", C.c_double), ("tc92", C.c_int32), ("h_maxit", C.c_int32),
                ("h_tol", C.c_double), ("kappa", C.c_double), ("leaf_size", C.c_int32),
                ("group_size", C.c_int32), ("walk_mode", C.c_int32), ("nbr_mode", C.c_int32),
                ("gravity", C.c_int32), ("hydro", C.c_int32), ("batch_size", C.c_int32),
                ("batch_mode", C.c_int32), ("grav_corr_literal", C.c_int32), ("soften_cells", C.c_int32),
                ("visc_form", C.c_int32), ("entropy", C.c_int32), ("xsph_eta", C.c_double),
                ("h_scheme", C.c_int32), ("h_weight", C.c_int32), ("balsara", C.c_int32),
                ("alpha_switch", C.c_int32), ("alpha_min", C.c_double), ("conduction", C.c_int32),
                ("alpha_u_min", C.c_double), ("period", C.c_double)]


class Run(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_gas", C.c_int64),
                ("x", D), ("y", D), ("z", D), ("vx", D), ("vy", D), ("vz", D), ("m", D), ("u", D),
                ("h_in", D), ("eps_in", D),
                ("h", D), ("nh", D), ("rho", D), ("omega", D), ("zeta", D), ("divv", D),
                ("eps", D), ("neps", D), ("ups", D), ("xi", D),
                ("ax", D), ("ay", D), ("az", D), ("pot", D), ("dudt", D), ("maxmu", D),
                ("cnt_node", I64), ("cnt_pair", I64), ("cnt_sph", I64), ("iters", I32),
                ("n_noconv", C.c_int64), ("sinks", I64), ("n_sinks", C.c_int64), ("cnt_soft", I64),
                ("divv_eps", D), ("t_phase", C.c_double * 4), ("xsph_x", D), ("xsph_y", D), ("xsph_z", D),
                ("vsig", D), ("alpha_in", D), ("alpha_u_in", D), ("dalpha", D), ("dalpha_u", D), ("curlx", D),
                ("curly", D), ("curlz", D), ("fbal", D), ("lapu", D)]


def eta_from_nnei(nnei: float) -> float:
    """eta such that N_nei = (4 pi / 3) (2 eta)^3 (Sect. 2.1, eps-n relation)."""
    return 0.5 * (3.0 * nnei / (4.0 * np.pi)) ** (1.0 / 3.0)


_LIB_PATH = None


def use_library(path: str):
    """Load the oracle from another build of the same source (for example
    one compiled for the host CPU); later calls go to it."""
    global _LIB, _LIB_PATH
    _LIB, _LIB_PATH = None, path
    return lib()


def lib():
    global _LIB
    if _LIB is None:
        path = _LIB_PATH or os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            from . import build as _b  # noqa: F401  (package-relative when imported as oracle.oracle)
            _b.build()
        L = C.CDLL(path)
        L.orc_compute_forces.argtypes = [C.POINTER(Params), C.POINTER(Run)]
        L.orc_compute_forces.restype = C.c_int
        L.orc_tree_build.argtypes = [C.c_int64, D, D, D, D, C.c_int32]
        L.orc_tree_build.restype = C.c_void_p
        L.orc_tree_free.argtypes = [C.c_void_p]
        L.orc_tree_nnodes.argtypes = [C.c_void_p]
        L.orc_tree_nnodes.restype = C.c_int64
        L.orc_tree_root.argtypes = [C.c_void_p, D, I32]
        L.orc_tree_keys.argtypes = [C.c_void_p, U64, I64]
        L.orc_tree_nodes.argtypes = [C.c_void_p, I32, U64, I64, I64, I64, I32, I64]
        L.orc_tree_moments.argtypes = [C.c_void_p, D, D, D, D, D, D, D, D]
        L.orc_tree_groups.argtypes = [C.c_void_p, C.c_int32, I64]
        L.orc_tree_groups.restype = C.c_int64
        L.orc_tree_batches.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32, I64, I64]
        L.orc_tree_batches.restype = C.c_int64
        L.orc_neighbours.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int64, D, D, D, D, C.c_int32,
                                     I64, I64, C.c_int64, C.c_double]
        L.orc_neighbours.restype = C.c_int64
        L.orc_potential_energy.argtypes = [C.c_int64, D, D, D, D, D, C.c_double]
        L.orc_potential_energy.restype = C.c_double
        L.orc_kick_drift.argtypes = [C.c_int64, C.c_int64, C.c_double, C.c_int32] + [D] * 22 + \
            [D, D, C.c_double, D, D, C.c_double, C.c_double]
        L.orc_ewald_exact.argtypes = [C.c_double] * 5 + [D]
        L.orc_ewald_interp.argtypes = [C.c_double] * 4 + [D]
        L.orc_timestep.argtypes = [C.POINTER(Params), C.c_int64, C.c_int64] + [D] * 12 + [C.c_double, D, D]
        L.orc_timestep.restype = C.c_double
        L.orc_timestep_each.argtypes = [C.POINTER(Params), C.c_int64, C.c_int64] + [D] * 12 + [C.c_double, D, D, D]
        L.orc_timestep_each.restype = C.c_double
        L.orc_diagnostics.argtypes = [C.c_int64, C.c_int64] + [D] * 10 + [D, C.c_double, C.c_int32]
        L.orc_eval_kernel.argtypes = [C.c_int, C.c_int64, D, D, D]
        L.orc_num_threads.restype = C.c_int
        L.orc_multipole_field.argtypes = [C.c_int64, D, D, D, D, C.c_double, C.c_double, C.c_double,
                                          C.c_int32, D, D]
        _LIB = L
    return _LIB


def _p(a, t=D):
    if a is None:
        return t()
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def params(**kw) -> Params:
    """Defaults: G = 1, theta = 0.5 with quadrupoles, adaptive softening with
    correction terms, 50 neighbours, gamma = 5/3, alpha = 1, beta = 2,
    eta_AV^2 = 0.01 hbar^2, TC92 gradient on, Newton tolerance 1e-6."""
    d = dict(G=1.0, theta=0.5, quadrupole=1, soft_mode=SOFT_ADAPTIVE,
             eta_h=eta_from_nnei(50.0), eta_eps=eta_from_nnei(50.0), gamma=5.0 / 3.0, alpha=1.0,
             beta=2.0, av_eps2=0.01, tc92=1, h_maxit=60, h_tol=1e-10, kappa=0.1, leaf_size=8,
             group_size=32, walk_mode=WALK_GROUP, nbr_mode=NBR_TREE, gravity=1, hydro=1, batch_size=64,
             batch_mode=0, grav_corr_literal=0, soften_cells=0, visc_form=VISC_MG, entropy=0, xsph_eta=0.0,
             h_scheme=H_LAGRANGIAN, h_weight=HW_NUMBER, balsara=0, alpha_switch=0, alpha_min=0.01,
             conduction=0, alpha_u_min=0.0, period=0.0)
    if "nnei" in kw:
        e = eta_from_nnei(kw.pop("nnei"))
        d["eta_h"] = d["eta_eps"] = e
    d.update(kw)
    return Params(**d)


KERNELS = {"W": 0, "dWdr": 1, "dWdh": 2, "tc92": 3, "phi": 4, "dphidr": 5, "dphideps": 6}


def kernel(name: str, r, h):
    r = _f64(np.atleast_1d(r))
    h = _f64(np.broadcast_to(np.atleast_1d(h), r.shape))
    out = np.empty_like(r)
    lib().orc_eval_kernel(KERNELS[name], r.size, _p(r), _p(h), _p(out))
    return out


def compute_forces(ic: dict, prm: Params, h_in=None, eps_in=None, vel=None, u=None, sinks=None, alpha=None,
                   alpha_u=None) -> dict:
    """Full oracle force evaluation on an initial-condition dict.

    ``vel``/``u`` override the velocities and internal energies used in the
    forces (the predicted values of the leapfrog)."""
    n, n_gas = int(ic["n"]), int(ic["n_gas"])
    x, y, z, m = (_f64(ic[k]) for k in ("x", "y", "z", "m"))
    if vel is None:
        vx, vy, vz = (_f64(ic[k]) for k in ("vx", "vy", "vz"))
    else:
        vx, vy, vz = (_f64(v) for v in vel)
    uu = _f64(ic["u"] if u is None else u)
    hin = None if h_in is None else _f64(h_in)
    ein = None if eps_in is None else _f64(eps_in)
    out = {k: np.zeros(n) for k in ("h", "nh", "rho", "omega", "zeta", "divv", "eps", "neps", "ups",
                                     "xi", "ax", "ay", "az", "pot", "dudt", "maxmu", "divv_eps", "xsph_x",
                                     "xsph_y", "xsph_z", "vsig", "dalpha", "dalpha_u", "curlx", "curly",
                                     "curlz", "fbal", "lapu")}
    cnt = {k: np.zeros(n, np.int64) for k in ("cnt_node", "cnt_pair", "cnt_sph", "cnt_soft")}
    snk = None if sinks is None else np.ascontiguousarray(sinks, dtype=np.int64)
    iters = np.zeros(n, np.int32)
    al = None if alpha is None else _f64(alpha)
    alu = None if alpha_u is None else _f64(alpha_u)
    r = Run(alpha_in=_p(al), alpha_u_in=_p(alu), n=n, n_gas=n_gas, x=_p(x), y=_p(y), z=_p(z), vx=_p(vx), vy=_p(vy), vz=_p(vz), m=_p(m),
            u=_p(uu), h_in=_p(hin), eps_in=_p(ein), iters=_p(iters, I32), sinks=_p(snk, I64),
            n_sinks=0 if snk is None else snk.size,
            **{k: _p(v) for k, v in out.items()}, **{k: _p(v, I64) for k, v in cnt.items()})
    rc = lib().orc_compute_forces(C.byref(prm), C.byref(r))
    if rc != 0:
        raise RuntimeError(f"orc_compute_forces failed ({rc})")
    out.update(cnt)
    out["iters"] = iters
    out["n_noconv"] = int(r.n_noconv)
    out["t_phase"] = dict(zip(("tree", "density", "gravity", "sph"), list(r.t_phase)))
    return out


def tree(ic_or_xyz, leaf_size: int, m=None, group_size: int | None = None, batch_size: int = 64,
         batch_mode: int = 0) -> dict:
    if isinstance(ic_or_xyz, dict):
        x, y, z = (_f64(ic_or_xyz[k]) for k in ("x", "y", "z"))
        m = ic_or_xyz.get("m") if m is None else m
    else:
        x, y, z = (_f64(a) for a in ic_or_xyz)
    n = x.size
    mm = None if m is None else _f64(m)
    L = lib()
    t = L.orc_tree_build(n, _p(x), _p(y), _p(z), _p(mm), leaf_size)
    if not t:
        raise RuntimeError("orc_tree_build failed")
    try:
        nn = L.orc_tree_nnodes(t)
        x0 = np.zeros(3)
        e = np.zeros(1, np.int32)
        L.orc_tree_root(t, _p(x0), _p(e, I32))
        keys = np.zeros(n, np.uint64)
        perm = np.zeros(n, np.int64)
        L.orc_tree_keys(t, _p(keys, U64), _p(perm, I64))
        level = np.zeros(nn, np.int32)
        prefix = np.zeros(nn, np.uint64)
        first, count, child, parent = (np.zeros(nn, np.int64) for _ in range(4))
        nchild = np.zeros(nn, np.int32)
        L.orc_tree_nodes(t, _p(level, I32), _p(prefix, U64), _p(first, I64), _p(count, I64),
                         _p(child, I64), _p(nchild, I32), _p(parent, I64))
        mass, delta, side = np.zeros(nn), np.zeros(nn), np.zeros(nn)
        com, centre, bmin, bmax = (np.zeros((nn, 3)) for _ in range(4))
        quad = np.zeros((nn, 6))
        L.orc_tree_moments(t, _p(mass), _p(com), _p(quad), _p(centre), _p(side), _p(delta),
                           _p(bmin), _p(bmax))
        out = dict(x0=x0, e=int(e[0]), keys=keys, perm=perm, level=level, prefix=prefix,
                   first=first, count=count, child=child, nchild=nchild, parent=parent, mass=mass,
                   com=com, quad=quad, centre=centre, side=side, delta=delta, bmin=bmin, bmax=bmax)
        if group_size is not None:
            ng = L.orc_tree_groups(t, group_size, I64())
            gn = np.zeros(max(ng, 1), np.int64)
            L.orc_tree_groups(t, group_size, _p(gn, I64))
            out["groups"] = gn[:ng]
            nb = L.orc_tree_batches(t, group_size, batch_size, batch_mode, I64(), I64())
            b0, b1 = np.zeros(max(nb, 1), np.int64), np.zeros(max(nb, 1), np.int64)
            L.orc_tree_batches(t, group_size, batch_size, batch_mode, _p(b0, I64), _p(b1, I64))
            out["batches"] = np.stack([b0[:nb], b1[:nb]], 1)
        return out
    finally:
        L.orc_tree_free(t)


def neighbours(kind: int, x, y, z, length, n_gas: int, mode: int = NBR_TREE, leaf_size: int = 8,
               cap: int | None = None, period: float = 0.0):
    """CSR neighbour sets (offsets[n+1], idx) -- see orc_neighbours."""
    x, y, z, length = (_f64(a) for a in (x, y, z, length))
    n = x.size
    off = np.zeros(n + 1, np.int64)
    if cap is None:
        cap = 256 * n + 1024
    idx = np.zeros(cap, np.int64)
    tot = lib().orc_neighbours(kind, mode, n, n_gas, _p(x), _p(y), _p(z), _p(length), leaf_size,
                               _p(off, I64), _p(idx, I64), cap, float(period))
    if tot < 0:
        return neighbours(kind, x, y, z, length, n_gas, mode, leaf_size, cap=int(off[-1]) + 1, period=period)
    return off, idx[:tot].copy()


def potential_energy(x, y, z, m, eps, G: float = 1.0) -> float:
    x, y, z, m, eps = (_f64(a) for a in (x, y, z, m, eps))
    return lib().orc_potential_energy(x.size, _p(x), _p(y), _p(z), _p(m), _p(eps), G)


def kick_drift(st: dict, dt: float, phase: int, acc, dudt, pred: dict | None = None,
               lengths: dict | None = None, xsph=None, alphas: dict | None = None, period: float = 0.0):
    """In-place KDK half step on a state dict (x, y, z, vx, vy, vz, u).

    ``lengths`` (phase 0): arrays "h" and "eps", updated in place along the
    drift from the divergences "divv" and "divv_eps" of the last force
    evaluation.  ``xsph`` (phase 0): the X-SPH velocity corrections (three
    arrays) added to the drift velocity of the gas.  ``alphas``: arrays
    "alpha", "alpha_u" (updated in place), their rates "dalpha", "dalpha_u"
    and floors "alpha_min", "alpha_u_min"."""
    ax, ay, az = (_f64(a) for a in acc)
    du = _f64(dudt)
    n, n_gas = int(st["n"]), int(st["n_gas"])
    vp = [None] * 4 if pred is None else [pred["vx"], pred["vy"], pred["vz"], pred["u"]]
    ln = [None] * 4
    if lengths is not None:
        ln = [lengths["h"], lengths["eps"], _f64(lengths["divv"]), _f64(lengths["divv_eps"])]
        for a in ln[:2]:
            assert a.dtype == np.float64 and a.flags.c_contiguous
    lib().orc_kick_drift(n, n_gas, dt, phase, *(_p(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "u")),
                         _p(ax), _p(ay), _p(az), _p(du), *(_p(v) for v in vp), *(_p(v) for v in ln),
                         *((_p(_f64(v)) for v in xsph) if xsph is not None else (D(), D(), D())),
                         *((_p(alphas["alpha"]), _p(_f64(alphas["dalpha"])), float(alphas["alpha_min"]),
                            _p(alphas["alpha_u"]), _p(_f64(alphas["dalpha_u"])), float(alphas["alpha_u_min"]))
                           if alphas is not None else (D(), D(), 0.0, D(), D(), 0.0)), float(period))


def ewald(x, y, z, L: float, omega: float | None = None) -> np.ndarray:
    """Ewald correction per unit mass at displacement (x, y, z): the sums
    (omega given) or the tabulated, interpolated form (omega None)."""
    out = np.zeros(3)
    if omega is None:
        lib().orc_ewald_interp(float(x), float(y), float(z), float(L), _p(out))
    else:
        lib().orc_ewald_exact(float(x), float(y), float(z), float(L), float(omega), _p(out))
    return out


def timestep(prm: Params, st: dict, out: dict, eta_dt: float = 0.1) -> float:
    n, n_gas = int(st["n"]), int(st["n_gas"])
    arrs = [st["vx"], st["vy"], st["vz"], st["u"], out["h"], out["eps"], out["ax"], out["ay"],
            out["az"], out["dudt"], out["divv"], out["maxmu"]]
    arrs = [_f64(a) for a in arrs]
    rho = _f64(out["rho"]) if "rho" in out else None
    al = _f64(st["alpha"]) if (prm.alpha_switch and st.get("alpha") is not None) else None
    return lib().orc_timestep(C.byref(prm), n, n_gas, *(_p(a) for a in arrs), eta_dt, _p(rho), _p(al))


def timestep_each(prm: Params, st: dict, out: dict, eta_dt: float = 0.1) -> np.ndarray:
    """Per-particle time-step criteria (Sect. 4.2), INFINITY where none applies."""
    n, n_gas = int(st["n"]), int(st["n_gas"])
    arrs = [st["vx"], st["vy"], st["vz"], st["u"], out["h"], out["eps"], out["ax"], out["ay"],
            out["az"], out["dudt"], out["divv"], out["maxmu"]]
    arrs = [_f64(a) for a in arrs]
    rho = _f64(out["rho"]) if "rho" in out else None
    al = _f64(st["alpha"]) if (prm.alpha_switch and st.get("alpha") is not None) else None
    dt = np.zeros(n)
    lib().orc_timestep_each(C.byref(prm), n, n_gas, *(_p(a) for a in arrs), eta_dt, _p(rho), _p(al), _p(dt))
    return dt


def diagnostics(st: dict, pot, rho=None, gamma: float = 5.0 / 3.0, entropy: bool = False) -> np.ndarray:
    """E_kin, E_th, V, P, L; with entropy, u holds A and E_th needs rho."""
    out = np.zeros(9)
    a = [_f64(st[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u")]
    p = _f64(pot)
    r = None if rho is None else _f64(rho)
    lib().orc_diagnostics(int(st["n"]), int(st["n_gas"]), *(_p(v) for v in a), _p(p), _p(out), _p(r),
                          float(gamma), int(bool(entropy)))
    return out


def num_threads() -> int:
    return int(lib().orc_num_threads())


def multipole_field(x, y, z, m, point, quadrupole: bool = True):
    """Acceleration and potential at ``point`` from the set's root-node
    expansion (monopole + optional quadrupole)."""
    x, y, z, m = (_f64(a) for a in (x, y, z, m))
    acc = np.zeros(3)
    pot = np.zeros(1)
    lib().orc_multipole_field(x.size, _p(x), _p(y), _p(z), _p(m), float(point[0]), float(point[1]),
                              float(point[2]), int(quadrupole), _p(acc), _p(pot))
    return acc, float(pot[0])
