"""Thin ctypes binding of the HIP library (``libtsph.so``, C ABI in
``include/tsph.h``).

Every function here only marshals arguments: device pointers come from torch
tensors (``data_ptr()``), streams from ``torch.cuda.current_stream()``.  The
computation runs in the library's HIP kernels.  Loading fails loudly when the
library is missing -- there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsph.so")

TSPH_OK, TSPH_EINVAL, TSPH_ENOMEM, TSPH_EHIP, TSPH_ECAPACITY, TSPH_ENOCONV, TSPH_EOVERFLOW = 0, -1, -2, -3, -4, -5, -6
SOFT_ADAPTIVE, SOFT_CONSTANT, SOFT_ADAPTIVE_NOCORR = 0, 1, 2
FP64, FP32_BULK = 0, 1
KD_FIRST, KD_SECOND = 0, 1
VISC_MG, VISC_SIGNAL = 0, 1
H_LAGRANGIAN, H_STANDARD = 0, 1
HW_NUMBER, HW_MASS = 0, 1
FLAG_NODE_CAPACITY, FLAG_STACK_OVERFLOW, FLAG_LIST_OVERFLOW, FLAG_NOCONV, FLAG_NONFINITE, FLAG_INTERNAL = (
    0x1, 0x2, 0x4, 0x8, 0x10, 0x20)
FLAG_HANDOFF_CAPACITY = 0x40
FLAG_PERIOD = 0x80
DBG_KEYS, DBG_PERM, DBG_NODES, DBG_NNODES, DBG_MOMENTS, DBG_GROUPS, DBG_NGROUPS, DBG_COUNTS, DBG_NBR, DBG_ROOT, \
    DBG_SOLVE, DBG_BATCHES, DBG_NBATCHES = range(13)
SOLVE_FIELDS = ("nh", "omega", "zeta", "divv", "neps", "ups", "xi", "maxmu", "divv_eps", "vsig", "duv", "xsph_sx",
                "xsph_sy", "xsph_sz", "curlx", "curly", "curlz", "fbal", "lapu")


class TsphError(RuntimeError):
    def __init__(self, fn, status, msg=""):
        super().__init__(f"{fn} failed with status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [("G", C.c_double), ("theta", C.c_double), ("quadrupole", C.c_int32), ("soft_mode", C.c_int32),
                ("eta_h", C.c_double), ("eta_eps", C.c_double), ("gamma", C.c_double), ("alpha", C.c_double),
                ("beta", C.c_double), ("av_eps2", C.c_double), ("tc92", C.c_int32), ("h_maxit", C.c_int32),
                ("h_tol", C.c_double), ("kappa", C.c_double), ("leaf_size", C.c_int32),
                ("group_size", C.c_int32), ("precision", C.c_int32), ("gravity", C.c_int32),
                ("hydro", C.c_int32), ("split_leaves", C.c_int32), ("eta_dt", C.c_double),
                ("max_members", C.c_int32), ("grav_corr_literal", C.c_int32), ("soften_cells", C.c_int32),
                ("visc_form", C.c_int32), ("entropy", C.c_int32), ("xsph_eta", C.c_double),
                ("h_scheme", C.c_int32), ("h_weight", C.c_int32), ("balsara", C.c_int32),
                ("alpha_switch", C.c_int32), ("conduction", C.c_int32), ("alpha_min", C.c_double),
                ("alpha_u_min", C.c_double), ("period", C.c_double)]


_P = C.c_void_p


class State(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_gas", C.c_int64),
                ("x", _P), ("y", _P), ("z", _P), ("vx", _P), ("vy", _P), ("vz", _P), ("m", _P), ("u", _P),
                ("vpx", _P), ("vpy", _P), ("vpz", _P), ("up", _P), ("h", _P), ("eps", _P),
                ("ax", _P), ("ay", _P), ("az", _P), ("dudt", _P), ("rho", _P), ("pot", _P),
                ("alpha", _P), ("alpha_u", _P)]


class Blocks(C.Structure):
    """tsph_blocks: individual power-of-two time-steps (see tsph.h)."""
    _fields_ = [("dt_max", C.c_double), ("max_level", C.c_int32), ("wake", C.c_int32), ("t", C.c_int64),
                ("n_active", C.c_int64), ("n_woken", C.c_int64), ("t0", _P), ("t1", _P), ("vsx", _P),
                ("vsy", _P), ("vsz", _P), ("us", _P)]


_LIB = None


def lib():
    """Load libtsph.so (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_0912_1786_amd/build.py "
                               "(or __graft_entry__.build()); there is no fallback path")
        # torch ships its own HIP runtime and loads it into the global symbol
        # scope; importing it first makes the library's HIP calls bind to that
        # same runtime, so torch's device pointers and streams are valid here.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        P, S = C.POINTER(Params), C.POINTER(State)
        sig = {
            "tsph_create": ([C.POINTER(C.c_void_p), C.c_int64, P], C.c_int),
            "tsph_destroy": ([_P], C.c_int),
            "tsph_set_params": ([_P, P], C.c_int),
            "tsph_default_params": ([P], None),
            "tsph_bytes_required": ([C.c_int64, P, C.POINTER(C.c_size_t)], C.c_int),
            "tsph_set_members": ([_P, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
            "tsph_build_tree": ([_P, S, _P], C.c_int),
            "tsph_compute_forces": ([_P, S, _P], C.c_int),
            "tsph_kick_drift": ([_P, S, C.c_double, C.c_int32, _P], C.c_int),
            "tsph_kick_drift_dt": ([_P, S, _P, C.c_int32, _P], C.c_int),
            "tsph_batch_step": ([_P, S, _P, _P], C.c_int),
            "tsph_carry_bytes": ([C.c_int64, C.POINTER(C.c_size_t)], C.c_int),
            "tsph_carry_save": ([_P, C.c_int64, _P, _P], C.c_int),
            "tsph_carry_load": ([_P, C.c_int64, _P, _P], C.c_int),
            "tsph_timestep": ([_P, S, _P, _P], C.c_int),
            "tsph_diagnostics": ([_P, S, _P, _P], C.c_int),
            "tsph_read_flags": ([_P, C.POINTER(C.c_uint32), C.POINTER(C.c_int64)], C.c_int),
            "tsph_take_flags_async": ([_P, _P, _P], C.c_int),
            "tsph_debug_lists": ([_P, C.c_int32], C.c_int),
            "tsph_timing": ([_P, C.c_int32], C.c_int),
            "tsph_phase_times": ([_P, C.POINTER(C.c_double), C.POINTER(C.c_int64)], C.c_int),
            "tsph_debug_export": ([_P, C.c_int32, _P, C.c_size_t, C.POINTER(C.c_size_t)], C.c_int),
            "tsph_debug_handoff_cap": ([_P, C.c_int64], C.c_int),
            "tsph_last_error": ([_P], C.c_char_p),
            "tsph_version": ([], C.c_char_p),
            "tsph_source_id": ([], C.c_char_p),
            "tsph_diagnostics_noalloc": ([S, C.c_int32, _P, _P, _P, _P], C.c_int),
            "tsph_noalloc_last_error": ([], C.c_char_p),
            "tsph_probe": ([C.c_int32, C.c_int64, _P, _P, _P, _P, C.POINTER(C.c_double)], C.c_int),
            "tsph_block_start": ([_P, S, C.POINTER(Blocks), _P], C.c_int),
            "tsph_block_advance": ([_P, S, C.POINTER(Blocks), _P], C.c_int),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        from .srcid import source_id
        built, here = L.tsph_source_id().decode(), source_id()
        if built != here:
            raise RuntimeError(f"{LIB_PATH} was built from other sources (id {built}) than those beside it "
                               f"(id {here}): rebuild it with paper_0912_1786_amd/build.py")
        _LIB = L
    return _LIB


EXPORTED = ("tsph_create", "tsph_destroy", "tsph_set_params", "tsph_default_params", "tsph_bytes_required",
            "tsph_set_members", "tsph_build_tree", "tsph_compute_forces", "tsph_kick_drift", "tsph_kick_drift_dt", "tsph_carry_bytes",
            "tsph_carry_save", "tsph_carry_load", "tsph_timestep", "tsph_diagnostics", "tsph_read_flags", "tsph_debug_lists", "tsph_debug_export", "tsph_last_error", "tsph_version",
            "tsph_timing", "tsph_phase_times", "tsph_probe", "tsph_debug_handoff_cap", "tsph_source_id",
            "tsph_diagnostics_noalloc", "tsph_noalloc_last_error", "tsph_batch_step", "tsph_block_start",
            "tsph_block_advance", "tsph_take_flags_async")
PHASES = ("tree", "density", "gravity", "sph", "finish")


def _check(fn, rc, ctx=None):
    if rc != TSPH_OK:
        # a NULL context reads the text of the last tsph_create failure
        m = lib().tsph_last_error(ctx)
        raise TsphError(fn, rc, m.decode() if m else "")


def eta_from_nnei(nnei: float) -> float:
    """eta with N_nei = (4 pi / 3) (2 eta)^3."""
    import math
    return 0.5 * (3.0 * nnei / (4.0 * math.pi)) ** (1.0 / 3.0)


def tsph_default_params(**kw) -> Params:
    p = Params()
    lib().tsph_default_params(C.byref(p))
    if "nnei" in kw:
        e = eta_from_nnei(kw.pop("nnei"))
        p.eta_h = p.eta_eps = e
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


def tsph_bytes_required(capacity_n: int, p: Params) -> int:
    b = C.c_size_t(0)
    _check("tsph_bytes_required", lib().tsph_bytes_required(int(capacity_n), C.byref(p), C.byref(b)))
    return int(b.value)


def tsph_create(capacity_n: int, p: Params):
    ctx = C.c_void_p()
    _check("tsph_create", lib().tsph_create(C.byref(ctx), int(capacity_n), C.byref(p)))
    return ctx


def tsph_destroy(ctx):
    _check("tsph_destroy", lib().tsph_destroy(ctx))


def tsph_set_params(ctx, p: Params):
    _check("tsph_set_params", lib().tsph_set_params(ctx, C.byref(p)), ctx)


def _stream(stream):
    if stream is None:
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return C.c_void_p(stream)
    return C.c_void_p(stream.cuda_stream)


def tsph_set_members(ctx, off, n_gas):
    """Several independent systems in one context: system k owns particles
    [off[k], off[k+1]) of the state, its first n_gas[k] being gas."""
    count = len(n_gas)
    if len(off) != count + 1:
        raise ValueError("off needs len(n_gas) + 1 entries")
    o = (C.c_int64 * (count + 1))(*[int(v) for v in off])
    g = (C.c_int64 * count)(*[int(v) for v in n_gas])
    _check("tsph_set_members", lib().tsph_set_members(ctx, count, o, g), ctx)


def tsph_build_tree(ctx, st: State, stream=None):
    _check("tsph_build_tree", lib().tsph_build_tree(ctx, C.byref(st), _stream(stream)), ctx)


def tsph_compute_forces(ctx, st: State, stream=None):
    _check("tsph_compute_forces", lib().tsph_compute_forces(ctx, C.byref(st), _stream(stream)), ctx)


def tsph_kick_drift(ctx, st: State, dt: float, phase: int, stream=None):
    _check("tsph_kick_drift", lib().tsph_kick_drift(ctx, C.byref(st), float(dt), int(phase), _stream(stream)), ctx)


def tsph_kick_drift_dt(ctx, st: State, dt_ptr: int, phase: int, stream=None):
    _check("tsph_kick_drift_dt",
           lib().tsph_kick_drift_dt(ctx, C.byref(st), C.c_void_p(dt_ptr), int(phase), _stream(stream)), ctx)


def tsph_batch_step(ctx, st: State, dt_ptr: int, stream=None):
    _check("tsph_batch_step", lib().tsph_batch_step(ctx, C.byref(st), C.c_void_p(dt_ptr), _stream(stream)), ctx)


def tsph_carry_bytes(n: int) -> int:
    b = C.c_size_t(0)
    _check("tsph_carry_bytes", lib().tsph_carry_bytes(int(n), C.byref(b)))
    return int(b.value)


def tsph_carry_save(ctx, n: int, dst_ptr: int, stream=None):
    _check("tsph_carry_save", lib().tsph_carry_save(ctx, int(n), C.c_void_p(dst_ptr), _stream(stream)), ctx)


def tsph_carry_load(ctx, n: int, src_ptr: int, stream=None):
    _check("tsph_carry_load", lib().tsph_carry_load(ctx, int(n), C.c_void_p(src_ptr), _stream(stream)), ctx)


def tsph_timestep(ctx, st: State, dt_ptr: int, stream=None):
    _check("tsph_timestep", lib().tsph_timestep(ctx, C.byref(st), C.c_void_p(dt_ptr), _stream(stream)), ctx)


def tsph_diagnostics(ctx, st: State, out_ptr: int, stream=None):
    _check("tsph_diagnostics", lib().tsph_diagnostics(ctx, C.byref(st), C.c_void_p(out_ptr), _stream(stream)), ctx)


NOALLOC_MAX_SYSTEMS = 910


def tsph_block_start(ctx, st: State, blk: Blocks, stream=None):
    _check("tsph_block_start", lib().tsph_block_start(ctx, C.byref(st), C.byref(blk), _stream(stream)), ctx)


def tsph_block_advance(ctx, st: State, blk: Blocks, stream=None):
    _check("tsph_block_advance", lib().tsph_block_advance(ctx, C.byref(st), C.byref(blk), _stream(stream)), ctx)


def tsph_diagnostics_noalloc(st: State, count: int, off_ptr: int, ngas_ptr: int, out_ptr: int, stream=None):
    """Context-free diagnostics into out_ptr (9 per system); off_ptr and
    ngas_ptr are device int64 tables (ignored for count = 1)."""
    rc = lib().tsph_diagnostics_noalloc(C.byref(st), int(count), C.c_void_p(off_ptr or None),
                                        C.c_void_p(ngas_ptr or None), C.c_void_p(out_ptr), _stream(stream))
    if rc != TSPH_OK:
        raise TsphError("tsph_diagnostics_noalloc", rc, lib().tsph_noalloc_last_error().decode())


def tsph_read_flags(ctx):
    f = C.c_uint32(0)
    nc = C.c_int64(0)
    _check("tsph_read_flags", lib().tsph_read_flags(ctx, C.byref(f), C.byref(nc)), ctx)
    return int(f.value), int(nc.value)


def tsph_take_flags_async(ctx, dst_ptr: int, stream=None):
    """Flag word and unconverged count (two uint32) to dst_ptr, then cleared,
    on the stream, without waiting."""
    _check("tsph_take_flags_async", lib().tsph_take_flags_async(ctx, C.c_void_p(dst_ptr), _stream(stream)), ctx)


def tsph_timing(ctx, enable: bool):
    _check("tsph_timing", lib().tsph_timing(ctx, int(bool(enable))), ctx)


def tsph_phase_times(ctx):
    """Summed milliseconds per phase (tree, density, gravity, sph, finish) and call count."""
    ms = (C.c_double * 5)()
    calls = C.c_int64(0)
    _check("tsph_phase_times", lib().tsph_phase_times(ctx, ms, C.byref(calls)), ctx)
    return dict(zip(PHASES, list(ms))), int(calls.value)


PROBE_FMA32, PROBE_FMA64, PROBE_TRIAD = 0, 1, 2


def tsph_probe(kind: int, n: int, a_ptr: int, b_ptr: int = 0, c_ptr: int = 0, stream=None) -> float:
    """Enqueue a machine probe (FMA chains or a stream triad) on the stream;
    returns the flops or bytes it performs."""
    work = C.c_double(0.0)
    _check("tsph_probe", lib().tsph_probe(int(kind), int(n), C.c_void_p(a_ptr), C.c_void_p(b_ptr),
                                          C.c_void_p(c_ptr), _stream(stream), C.byref(work)))
    return work.value


def tsph_debug_lists(ctx, max_per_particle: int):
    _check("tsph_debug_lists", lib().tsph_debug_lists(ctx, int(max_per_particle)), ctx)


def tsph_debug_export(ctx, what: int, nbytes: int):
    """Copy a debug array to a host bytes buffer (see TSPH_DBG_* in tsph.h)."""
    buf = C.create_string_buffer(max(int(nbytes), 8))
    w = C.c_size_t(0)
    _check("tsph_debug_export", lib().tsph_debug_export(ctx, int(what), buf, len(buf), C.byref(w)), ctx)
    return buf.raw[:w.value]


def tsph_debug_handoff_cap(ctx, items: int):
    _check("tsph_debug_handoff_cap", lib().tsph_debug_handoff_cap(ctx, int(items)), ctx)


def tsph_last_error(ctx) -> str:
    m = lib().tsph_last_error(ctx)
    return m.decode() if m else ""


def tsph_version() -> str:
    return lib().tsph_version().decode()


# ---------------------------------------------------------------------------
# convenience: a particle set held in torch device tensors
# ---------------------------------------------------------------------------
def concat_ics(ics):
    """One initial-condition dict holding the systems of ``ics`` back to back
    (each with its gas first, as the inputs generate them), and the member
    table [(n, n_gas), ...] for Simulation(members=...)."""
    import numpy as np
    keys = ("x", "y", "z", "vx", "vy", "vz", "m", "u")
    out = {k: np.concatenate([np.asarray(ic[k], dtype=np.float64) for ic in ics]) for k in keys}
    out["n"] = int(sum(int(ic["n"]) for ic in ics))
    out["n_gas"] = int(sum(int(ic["n_gas"]) for ic in ics))
    return out, [(int(ic["n"]), int(ic["n_gas"])) for ic in ics]


class Simulation:
    """Caller-owned FP64 device arrays for one particle system plus a context.

    ``ic`` is a dict from :mod:`paper_0912_1786_amd.inputs`.  The predicted
    velocity/energy arrays start as copies of v and u (first evaluation).
    With ``members`` = [(n, n_gas), ...] (see concat_ics) the arrays hold
    that many independent systems back to back in one context; timestep()
    and diagnostics() then return one entry per system.  With ``ctx`` and
    ``bufs`` (a context of capacity >= n and one device float64 tensor of
    length >= n per name of FIELDS, plus "dt" and "diag") the system lives
    in that borrowed memory: nothing is allocated and close() leaves it.
    """

    FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "vpx", "vpy", "vpz", "up", "h", "eps", "ax", "ay", "az",
              "dudt", "rho", "pot", "alpha", "alpha_u")

    def __init__(self, ic: dict, params: Params | None = None, capacity: int | None = None, device: str = "cuda",
                 want_pot: bool = True, eps_const=None, members=None, ctx=None, bufs=None, fill: bool = True):
        import torch
        self.torch = torch
        self.n = int(ic["n"])
        self.n_gas = int(ic["n_gas"])
        self.params = Params.from_buffer_copy(params if params is not None else tsph_default_params())
        self.count = 1 if members is None else len(members)
        self.off = [0]
        for nk, _ in (members or [(self.n, self.n_gas)]):
            self.off.append(self.off[-1] + int(nk))
        if self.off[-1] != self.n:
            raise ValueError("the members do not add up to n")
        if members is not None:
            self.params.max_members = max(int(self.params.max_members), self.count)
        dev = torch.device(device)
        n = self.n
        if bufs is not None:
            if ctx is None:
                raise ValueError("bufs need the context they belong to")
            if fill:
                t = lambda a, k: bufs[k][:n].copy_(torch.as_tensor(a, dtype=torch.float64), non_blocking=False)
                z = lambda k: bufs[k][:n].zero_()
            else:
                # bind the buffers as they are: the caller restores the state
                t = lambda a, k: bufs[k][:n]
                z = lambda k: bufs[k][:n]
        else:
            t = lambda a, k: torch.as_tensor(a, dtype=torch.float64).to(dev).contiguous()
            z = lambda k: torch.zeros(n, dtype=torch.float64, device=dev)
        self.a = {}
        for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u"):
            self.a[k] = t(ic[k], k)
        for k, src in (("vpx", "vx"), ("vpy", "vy"), ("vpz", "vz"), ("up", "u")):
            if bufs is not None:
                self.a[k] = bufs[k][:n].copy_(self.a[src]) if fill else bufs[k][:n]
            else:
                self.a[k] = self.a[src].clone()
        self.a["h"] = z("h")
        self.a["eps"] = z("eps") if eps_const is None else t(eps_const, "eps")
        for k in ("ax", "ay", "az", "dudt", "rho"):
            self.a[k] = z(k)
        # dissipation coefficients: alpha from the parameters, alpha_u zero,
        # unless the initial conditions give them
        if "alpha" in ic:
            self.a["alpha"] = t(ic["alpha"], "alpha")
        else:
            self.a["alpha"] = z("alpha").fill_(self.params.alpha) if fill else z("alpha")
        self.a["alpha_u"] = t(ic["alpha_u"], "alpha_u") if "alpha_u" in ic else z("alpha_u")
        self.a["pot"] = z("pot") if want_pot else None
        self.owns_ctx = ctx is None
        self.ctx = ctx if ctx is not None else tsph_create(capacity or self.n, self.params)
        if members is not None:
            try:
                tsph_set_members(self.ctx, self.off, [g for _, g in members])
            except Exception:
                self.close()
                raise
        self.state = self._state()
        if bufs is not None:
            self.diag_buf = bufs["diag"][:9 * self.count]
            self.dt_buf = bufs["dt"][:self.count]
        else:
            self.diag_buf = torch.zeros(9 * self.count, dtype=torch.float64, device=dev)
            self.dt_buf = torch.zeros(self.count, dtype=torch.float64, device=dev)

    def _state(self) -> State:
        st = State()
        st.n, st.n_gas = self.n, self.n_gas
        for k in self.FIELDS:
            v = self.a[k]
            setattr(st, k, None if v is None else v.data_ptr())
        return st

    def compute_forces(self, stream=None):
        tsph_compute_forces(self.ctx, self.state, stream)

    # ---- individual power-of-two time-steps ---------------------------------
    def block_start(self, dt_max: float, max_level: int, wake: int = 4, stream=None):
        """First system time of a run with individual time-steps: force pass
        over all particles, steps chosen, opening kicks."""
        torch = self.torch
        dev = self.a["x"].device
        n = self.n
        self.blk_a = {k: torch.zeros(n, dtype=torch.int32, device=dev) for k in ("t0", "t1")}
        for k in ("vsx", "vsy", "vsz", "us"):
            self.blk_a[k] = torch.zeros(n, dtype=torch.float64, device=dev)
        b = Blocks()
        b.dt_max, b.max_level, b.wake = float(dt_max), int(max_level), int(wake)
        for k, v in self.blk_a.items():
            setattr(b, k, v.data_ptr())
        self.blk = b
        tsph_block_start(self.ctx, self.state, b, stream)

    def block_advance(self, stream=None):
        """Advance to the next system time; returns (t, n_active, n_woken)."""
        tsph_block_advance(self.ctx, self.state, self.blk, stream)
        return int(self.blk.t), int(self.blk.n_active), int(self.blk.n_woken)

    def block_host(self, key: str):
        """Host copy of a block-step array: t0, t1 (ticks), vsx, vsy, vsz, us."""
        self.torch.cuda.synchronize()
        return self.blk_a[key].cpu().numpy()

    def kick_drift(self, dt: float, phase: int, stream=None):
        tsph_kick_drift(self.ctx, self.state, dt, phase, stream)

    def timestep(self, stream=None):
        """The time-step of the last force pass: a float, or one per system."""
        tsph_timestep(self.ctx, self.state, self.dt_buf.data_ptr(), stream)
        v = self.dt_buf.cpu().numpy()
        return float(v[0]) if self.count == 1 else v

    def diagnostics(self, stream=None):
        """E_kin, E_th, V, P, L: shape (9,), or (systems, 9)."""
        tsph_diagnostics(self.ctx, self.state, self.diag_buf.data_ptr(), stream)
        v = self.diag_buf.cpu().numpy()
        return v if self.count == 1 else v.reshape(self.count, 9)

    def member(self, k: int, key: str):
        """Host copy of array `key` of system k."""
        return self.a[key][self.off[k]:self.off[k + 1]].cpu().numpy()

    def step(self, dt: float, stream=None):
        """One KDK step; assumes forces of the current state are present."""
        self.kick_drift(dt, KD_FIRST, stream)
        self.compute_forces(stream)
        self.kick_drift(dt, KD_SECOND, stream)

    def carry(self):
        """Host copy of the context's carry to the next step (see tsph_carry_save)."""
        torch = self.torch
        buf = torch.empty(tsph_carry_bytes(self.n) // 8, dtype=torch.float64, device=self.a["x"].device)
        tsph_carry_save(self.ctx, self.n, buf.data_ptr())
        torch.cuda.current_stream().synchronize()
        return buf.cpu().numpy()

    def load_carry(self, host):
        torch = self.torch
        buf = torch.from_numpy(host).to(self.a["x"].device)
        tsph_carry_load(self.ctx, self.n, buf.data_ptr())
        torch.cuda.current_stream().synchronize()

    def device_step(self, stream=None):
        """One KDK step of every system held, each with its own global
        time-step taken and used on the device (tsph_batch_step: no host
        round trip; capturable in a HIP graph)."""
        tsph_batch_step(self.ctx, self.state, self.dt_buf.data_ptr(), stream)

    def flags(self):
        return tsph_read_flags(self.ctx)

    def host(self, k):
        return self.a[k].cpu().numpy()

    def export(self, what: int, dtype, count: int):
        import numpy as np
        raw = tsph_debug_export(self.ctx, what, count * np.dtype(dtype).itemsize)
        return np.frombuffer(raw, dtype=dtype).copy()

    def close(self):
        if self.ctx is not None:
            if getattr(self, "owns_ctx", True):
                tsph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
