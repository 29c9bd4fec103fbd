"""Python binding of the C ABI in ``include/fte.h`` (argument marshalling only).

Every step of the path runs in the HIP kernels of ``libfte.so``; this module
only converts plain workload descriptions into the C structures, owns the
device buffers as torch tensors (torch is used for device memory and streams),
and forwards calls.  If the library is missing the import fails: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FTE_LIB_PATH") or os.path.join(_HERE, "libfte.so")

FTE_OK, FTE_EINVAL, FTE_ESTATE, FTE_ENOMEM, FTE_EDEVICE, FTE_ERANGE = 0, -1, -2, -3, -4, -5
FTE_FP64, FTE_MIXED = 0, 1
DMM = {"iso": 0, "eq5": 1, "power_q": 2}
MAX_OBS = 8
RECORD_STRIDE = 10        # fields 0-9 (no kappa_perp)
RECORD_STRIDE_KPERP = 13  # fields 0-12
RECORD_FIELDS = 13
STATUS = {"active": 0, "absorbed_in": 1, "absorbed_out": 2, "out_of_domain": 3, "numeric": 4, "done": 5}
MAX_RUNS = 64
SYMBOLS = ["fte_create", "fte_destroy", "fte_last_error", "fte_query_sizes", "fte_bind_buffers", "fte_load_grid",
           "fte_inject", "fte_step_n", "fte_bin_observers", "fte_read_hist", "fte_get_stats", "fte_read_particles",
           "fte_set_launch", "fte_reset", "fte_set_timing", "fte_bin_smoothed", "fte_grad", "fte_read_tangents",
           "fte_state_size", "fte_save_state", "fte_load_state", "fte_autotune", "fte_bin_steady",
           "fte_load_snapshot", "fte_set_record_tile", "fte_plan_snapshot", "fte_bin_observers_static",
           "fte_capture_begin", "fte_capture_end", "fte_graph_launch", "fte_graph_destroy",
           "fte_set_lds_histogram"]
TANGENT_COLS = 11         # d(x, y, z, mu, lnp)/d lambda_ref, the same for kperp_ratio, d ln w / d gamma_inj


class fte_observer(C.Structure):
    _fields_ = [("r", C.c_double), ("theta", C.c_double), ("phi", C.c_double),
                ("dr", C.c_double), ("dtheta", C.c_double), ("dphi", C.c_double),
                ("n_phi", C.c_int), ("omega", C.c_double)]


class fte_run(C.Structure):
    _fields_ = [("lambda_ref", C.c_double), ("kperp_ratio", C.c_double), ("n_steps", C.c_uint64)]


class fte_params(C.Structure):
    _fields_ = [("mass", C.c_double), ("dmm_model", C.c_int), ("dmm_norm", C.c_int),
                ("lambda_ref", C.c_double), ("p_ref", C.c_double), ("alpha", C.c_double),
                ("q", C.c_double), ("eps", C.c_double), ("mu_floor", C.c_double),
                ("kperp_ratio", C.c_double), ("lambda_perp", C.c_double),
                ("dt", C.c_double), ("t0", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double),
                ("seed", C.c_uint64), ("run_id", C.c_int), ("precision", C.c_int),
                ("n_obs", C.c_int), ("obs", fte_observer * MAX_OBS),
                ("e_min", C.c_double), ("dlne", C.c_double), ("n_e", C.c_int),
                ("t_ref", C.c_double), ("dT", C.c_double), ("n_t", C.c_int), ("n_batch", C.c_int),
                ("sigma_x", C.c_double), ("sigma_lne", C.c_double), ("sigma_t", C.c_double), ("grad", C.c_int),
                ("n_runs", C.c_int), ("runs", C.POINTER(fte_run)),
                ("kink_sigma", C.c_double)]


class fte_grid_desc(C.Structure):
    _fields_ = [("xi_map", C.c_int), ("r_lo", C.c_double), ("dxi", C.c_double),
                ("th_lo", C.c_double), ("dth", C.c_double), ("ph_lo", C.c_double), ("dph", C.c_double),
                ("phi_periodic", C.c_int), ("n1", C.c_int * 3), ("bx", C.c_int * 3), ("n_levels", C.c_int),
                ("n_leaves", C.c_int), ("leaves", C.POINTER(C.c_int32)), ("n_snap", C.c_int),
                ("t_s0", C.c_double), ("dt_s", C.c_double), ("n_slots", C.c_int), ("n_pool", C.c_int)]


class fte_injection(C.Structure):
    _fields_ = [("r", C.c_double), ("th_lo", C.c_double), ("th_hi", C.c_double), ("ph_lo", C.c_double),
                ("ph_hi", C.c_double), ("e_lo", C.c_double), ("e_hi", C.c_double), ("gamma_inj", C.c_double),
                ("w0", C.c_double), ("r_weight", C.c_int), ("r_ref", C.c_double), ("pid0", C.c_uint64),
                ("n_total", C.c_uint64), ("k0", C.c_uint32), ("n_inj_steps", C.c_uint32), ("run", C.c_int),
                ("region", C.c_int), ("r_hi", C.c_double), ("divv_max", C.c_double), ("max_tries", C.c_uint32)]


class fte_sizes(C.Structure):
    _fields_ = [("grid_bytes", C.c_uint64), ("index_bytes", C.c_uint64), ("state_bytes", C.c_uint64),
                ("hist_bytes", C.c_uint64), ("work_bytes", C.c_uint64), ("tangent_bytes", C.c_uint64)]


class fte_buffers(C.Structure):
    _fields_ = [("grid", C.c_void_p), ("index", C.c_void_p), ("state_a", C.c_void_p), ("state_b", C.c_void_p),
                ("hist", C.c_void_p), ("work", C.c_void_p), ("tangent_a", C.c_void_p), ("tangent_b", C.c_void_p)]


class fte_stats(C.Structure):
    _fields_ = [("n_live", C.c_uint64), ("n_injected", C.c_uint64), ("particle_steps", C.c_uint64),
                ("n_retired", C.c_uint64 * 6), ("w_injected", C.c_double), ("w_retired", C.c_double * 6),
                ("global_step", C.c_uint64), ("device_flags", C.c_uint32), ("step_launches", C.c_uint32),
                ("step_kernel_ms", C.c_double)]


_lib = None


def lib():
    """Load libfte.so (built by ``paper_2404_12164_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2404_12164_amd.build")
        L = C.CDLL(LIB_PATH)
        vp, u64, u32 = C.c_void_p, C.c_uint64, C.c_uint32
        dp = C.POINTER(C.c_double)
        L.fte_create.argtypes = [C.POINTER(vp), C.POINTER(fte_params)]
        L.fte_destroy.argtypes = [vp]
        L.fte_destroy.restype = None
        L.fte_last_error.argtypes = [vp]
        L.fte_last_error.restype = C.c_char_p
        L.fte_query_sizes.argtypes = [C.POINTER(fte_params), C.POINTER(fte_grid_desc), u64, C.POINTER(fte_sizes)]
        L.fte_bind_buffers.argtypes = [vp, C.POINTER(fte_grid_desc), u64, C.POINTER(fte_buffers)]
        L.fte_load_grid.argtypes = [vp, vp, vp]
        L.fte_inject.argtypes = [vp, C.POINTER(fte_injection), u64, u64, vp]
        L.fte_step_n.argtypes = [vp, u32, vp]
        L.fte_bin_observers.argtypes = [vp, dp, dp, C.c_int, vp]
        L.fte_bin_observers_static.argtypes = [vp, dp, dp, C.c_int, vp]
        L.fte_read_hist.argtypes = [vp, dp, dp, vp]
        L.fte_get_stats.argtypes = [vp, C.POINTER(fte_stats), vp]
        L.fte_read_particles.argtypes = [vp, dp, dp, dp, dp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint32),
                                         C.POINTER(C.c_int32), u64, C.POINTER(C.c_uint64), vp]
        L.fte_set_launch.argtypes = [vp, C.c_int, C.c_int, C.c_int, C.c_int]
        L.fte_set_record_tile.argtypes = [vp, C.c_int]
        L.fte_plan_snapshot.argtypes = [vp, C.c_int, C.POINTER(fte_injection), C.c_int, C.c_double,
                                        C.POINTER(C.c_int32), u64, C.POINTER(C.c_uint64), vp]
        L.fte_reset.argtypes = [vp, vp]
        L.fte_set_timing.argtypes = [vp, C.c_int]
        L.fte_bin_smoothed.argtypes = [vp, dp, dp, vp]
        L.fte_grad.argtypes = [vp, dp, dp, vp]
        L.fte_read_tangents.argtypes = [vp, dp, u64, C.POINTER(C.c_uint64), vp]
        L.fte_state_size.argtypes = [vp, C.POINTER(C.c_uint64), vp]
        L.fte_save_state.argtypes = [vp, vp, u64, vp]
        L.fte_load_state.argtypes = [vp, vp, u64, vp]
        L.fte_autotune.argtypes = [vp, u32, C.POINTER(C.c_int), vp]
        L.fte_bin_steady.argtypes = [vp, dp, dp, vp]
        L.fte_load_snapshot.argtypes = [vp, C.c_int, C.POINTER(vp), vp]
        L.fte_set_lds_histogram.argtypes = [vp, C.c_int]
        L.fte_capture_begin.argtypes = [vp, vp]
        L.fte_capture_end.argtypes = [vp, vp, C.POINTER(vp)]
        L.fte_graph_launch.argtypes = [vp, vp, vp]
        L.fte_graph_destroy.argtypes = [vp]
        L.fte_graph_destroy.restype = None
        for name in SYMBOLS:
            if name not in ("fte_destroy", "fte_last_error", "fte_graph_destroy"):
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


class Graph:
    """A recorded launch graph (fte_capture_end); free it with close()."""

    def __init__(self, handle):
        self.handle = handle

    def close(self):
        if self.handle:
            fte_graph_destroy(self.handle)
            self.handle = None


class FteError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"fte status {status}: {msg}")
        self.status = status


# ----------------------------------------------------------------------------
# marshalling of plain workload descriptions
# ----------------------------------------------------------------------------
def make_params(p: dict) -> fte_params:
    o = fte_params()
    o.mass = p["mass"]
    dm = p.get("dmm_model", "power_q")
    o.dmm_model = DMM[dm] if isinstance(dm, str) else int(dm)
    o.dmm_norm = int(p.get("dmm_norm", 0))
    o.lambda_ref = p["lambda_ref"]
    o.p_ref = p.get("p_ref", 1.0)
    o.alpha = p.get("alpha", 0.0)
    o.q = p.get("q", 5.0 / 3.0)
    o.eps = p.get("eps", 0.0)
    o.mu_floor = p.get("mu_floor", 1e-4)
    o.kperp_ratio = p.get("kperp_ratio", 0.0)
    o.lambda_perp = p.get("lambda_perp", 0.0)
    o.dt = p["dt"]
    o.t0 = p.get("t0", 0.0)
    o.r_in = p.get("r_in", 0.0)
    o.r_out = p.get("r_out", 1e300)
    o.seed = int(p.get("seed", 0))
    o.run_id = int(p.get("run_id", 0))
    prec = p.get("precision", "fp64")
    o.precision = {"fp64": FTE_FP64, "mixed": FTE_MIXED}[prec] if isinstance(prec, str) else int(prec)
    obs = p.get("observers", [])
    o.n_obs = len(obs)
    for i, ob in enumerate(obs):
        o.obs[i] = fte_observer(*[float(v) for v in ob[:6]], int(ob[6]) if len(ob) > 6 else 1,
                                float(ob[7]) if len(ob) > 7 else 0.0)
    o.e_min = p.get("e_min", 1.0)
    o.dlne = p.get("dlne", 1.0)
    o.n_e = int(p.get("n_e", 1))
    o.t_ref = p.get("t_ref", 0.0)
    o.dT = p.get("dT", 1.0)
    o.n_t = int(p.get("n_t", 1))
    o.n_batch = int(p.get("n_batch", 32))
    sm = p.get("smoothing")
    if sm:
        o.sigma_x, o.sigma_lne, o.sigma_t = sm["sigma_x"], sm["sigma_lne"], sm["sigma_t"]
    o.grad = int(p.get("grad", 0))
    runs = p.get("runs") or []
    o.n_runs = len(runs)
    if runs:
        arr = (fte_run * len(runs))()
        for i, r in enumerate(runs):
            arr[i] = fte_run(float(r["lambda_ref"]), float(r.get("kperp_ratio", 0.0)), int(r["n_steps"]))
        o.runs = C.cast(arr, C.POINTER(fte_run))
        o._runs_keep = arr          # the C call reads the table; keep it alive with the struct
    o.kink_sigma = p.get("kink_sigma", 0.0)
    return o


def make_grid_desc(g: dict):
    leaves = np.ascontiguousarray(g["leaves"], dtype=np.int32)
    d = fte_grid_desc()
    d.xi_map = int(g["xi_map"])
    d.r_lo, d.dxi = g["r_lo"], g["dxi"]
    d.th_lo, d.dth = g["th_lo"], g["dth"]
    d.ph_lo, d.dph = g["ph_lo"], g["dph"]
    d.phi_periodic = int(g["phi_periodic"])
    for a in range(3):
        d.n1[a] = int(g["n1"][a])
        d.bx[a] = int(g["bx"][a])
    d.n_levels = int(g["n_levels"])
    d.n_leaves = int(leaves.shape[0])
    d.leaves = leaves.ctypes.data_as(C.POINTER(C.c_int32))
    d.n_snap = int(g["n_snap"])
    d.t_s0 = g.get("t_s0", 0.0)
    d.dt_s = g.get("dt_s", 1.0)
    d.n_slots = int(g.get("n_slots", 0))
    d.n_pool = int(g.get("n_pool", 0))
    return d, leaves


def make_injection(inj: dict) -> fte_injection:
    o = fte_injection()
    o.r = inj["r"]
    o.th_lo, o.th_hi = inj["th_lo"], inj["th_hi"]
    o.ph_lo, o.ph_hi = inj["ph_lo"], inj["ph_hi"]
    o.e_lo = inj["e_lo"]
    o.e_hi = inj.get("e_hi", inj["e_lo"])
    o.gamma_inj = inj.get("gamma_inj", 1.0)
    o.w0 = inj.get("w0", 1.0)
    o.r_weight = int(inj.get("r_weight", 0))
    o.r_ref = inj.get("r_ref", 1.0)
    o.pid0 = int(inj.get("pid0", 0))
    o.n_total = int(inj["n_total"])
    o.k0 = int(inj.get("k0", 0))
    o.n_inj_steps = int(inj.get("n_inj_steps", 0))
    o.run = int(inj.get("run", 0))
    o.region = int(inj.get("region", 0))
    o.r_hi = inj.get("r_hi", inj["r"])
    o.divv_max = inj.get("divv_max", 0.0)
    o.max_tries = int(inj.get("max_tries", 4096))
    return o


# ----------------------------------------------------------------------------
# thin wrappers with the C names
# ----------------------------------------------------------------------------
def _check(ctx, st):
    if st != FTE_OK:
        msg = lib().fte_last_error(ctx).decode() if ctx else ""
        raise FteError(st, msg)


def fte_create(params: dict):
    h = C.c_void_p()
    pp = make_params(params)
    st = lib().fte_create(C.byref(h), C.byref(pp))
    if st != FTE_OK:
        raise FteError(st, "invalid parameters")
    return h


def fte_destroy(ctx):
    lib().fte_destroy(ctx)


def fte_query_sizes(params: dict, grid: dict, n_max: int) -> fte_sizes:
    pp = make_params(params)
    gd, _keep = make_grid_desc(grid)
    out = fte_sizes()
    st = lib().fte_query_sizes(C.byref(pp), C.byref(gd), int(n_max), C.byref(out))
    if st != FTE_OK:
        raise FteError(st, "invalid parameters or grid")
    return out


def fte_bind_buffers(ctx, grid: dict, n_max: int, bufs: fte_buffers):
    gd, _keep = make_grid_desc(grid)
    _check(ctx, lib().fte_bind_buffers(ctx, C.byref(gd), int(n_max), C.byref(bufs)))


def fte_load_grid(ctx, vb_sph_ptr: int, stream: int):
    _check(ctx, lib().fte_load_grid(ctx, C.c_void_p(vb_sph_ptr), C.c_void_p(stream)))


def fte_load_snapshot(ctx, k: int, ptrs, stream: int):
    """ptrs: five device addresses (0 for none) of snapshots k-2 .. k+2."""
    arr = (C.c_void_p * 5)(*[C.c_void_p(int(v)) if v else None for v in ptrs])
    _check(ctx, lib().fte_load_snapshot(ctx, int(k), arr, C.c_void_p(stream)))


def fte_plan_snapshot(ctx, k: int, sources, wind_speed_max: float, n_leaves: int, stream: int):
    """Leaves snapshot k's slot holds (a streamed subset): returns the ids of
    the leaves whose input the load reads and the counts (gather, held,
    input)."""
    arr = (fte_injection * max(len(sources), 1))(*[make_injection(q) for q in sources])
    out = np.zeros(n_leaves, dtype=np.int32)
    counts = (C.c_uint64 * 3)()
    _check(ctx, lib().fte_plan_snapshot(ctx, int(k), arr, len(sources), float(wind_speed_max),
                                        out.ctypes.data_as(C.POINTER(C.c_int32)), n_leaves, counts,
                                        C.c_void_p(stream)))
    return out[: counts[2]].copy(), (int(counts[0]), int(counts[1]), int(counts[2]))


def fte_inject(ctx, inj: dict, n: int, first_pid: int, stream: int):
    io = make_injection(inj)
    _check(ctx, lib().fte_inject(ctx, C.byref(io), int(n), int(first_pid), C.c_void_p(stream)))


def fte_step_n(ctx, n_steps: int, stream: int):
    _check(ctx, lib().fte_step_n(ctx, int(n_steps), C.c_void_p(stream)))


def fte_bin_observers(ctx, shape, reset: bool, stream: int):
    n = int(np.prod(shape))
    j = np.zeros(max(n, 1))
    s = np.zeros(max(n, 1))
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_bin_observers(ctx, j.ctypes.data_as(dp), s.ctypes.data_as(dp), int(bool(reset)),
                                        C.c_void_p(stream)))
    return j[:n].reshape(shape), s[:n].reshape(shape)


def fte_bin_observers_static(ctx, shape, reset: bool, stream: int):
    """fte_bin_observers through the library's fixed device scratch (no
    allocation)."""
    n = int(np.prod(shape))
    j = np.zeros(max(n, 1))
    s = np.zeros(max(n, 1))
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_bin_observers_static(ctx, j.ctypes.data_as(dp), s.ctypes.data_as(dp), int(bool(reset)),
                                               C.c_void_p(stream)))
    return j[:n].reshape(shape), s[:n].reshape(shape)


def fte_bin_steady(ctx, shape, stream: int):
    n = int(np.prod(shape))
    j = np.zeros(max(n, 1))
    s = np.zeros(max(n, 1))
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_bin_steady(ctx, j.ctypes.data_as(dp), s.ctypes.data_as(dp), C.c_void_p(stream)))
    return j[:n].reshape(shape), s[:n].reshape(shape)


def obs_bins(params: dict) -> int:
    """Observer bins: each observer (r, theta, phi, dr, dtheta, dphi[, n_phi[,
    omega]]) covers n_phi longitude bins."""
    return sum(int(ob[6]) if len(ob) > 6 and int(ob[6]) > 1 else 1 for ob in params.get("observers", []))


def fte_read_hist(ctx, n: int, stream: int, n_runs: int = 0):
    h = np.zeros(max(n, 1))
    w = np.zeros(max(n_runs, 1))
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_read_hist(ctx, h.ctypes.data_as(dp), w.ctypes.data_as(dp), C.c_void_p(stream)))
    return h[:n], (w if n_runs > 0 else float(w[0]))


def fte_get_stats(ctx, stream: int) -> fte_stats:
    out = fte_stats()
    _check(ctx, lib().fte_get_stats(ctx, C.byref(out), C.c_void_p(stream)))
    return out


def fte_read_particles(ctx, cap: int, stream: int) -> dict:
    x = np.zeros((cap, 3))
    mu = np.zeros(cap)
    lnp = np.zeros(cap)
    w = np.zeros(cap)
    pid = np.zeros(cap, dtype=np.uint64)
    kinj = np.zeros(cap, dtype=np.uint32)
    status = np.zeros(cap, dtype=np.int32)
    n = C.c_uint64()
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_read_particles(ctx, x.ctypes.data_as(dp), mu.ctypes.data_as(dp), lnp.ctypes.data_as(dp),
                                         w.ctypes.data_as(dp), pid.ctypes.data_as(C.POINTER(C.c_uint64)),
                                         kinj.ctypes.data_as(C.POINTER(C.c_uint32)),
                                         status.ctypes.data_as(C.POINTER(C.c_int32)), int(cap), C.byref(n),
                                         C.c_void_p(stream)))
    k = n.value
    return dict(x=x[:k], mu=mu[:k], lnp=lnp[:k], w=w[:k], pid=pid[:k], kinj=kinj[:k], status=status[:k])


def fte_bin_smoothed(ctx, shape, grad: bool, stream: int):
    n = int(np.prod(shape))
    J = np.zeros(max(n, 1))
    dJ = np.zeros((3, max(n, 1))) if grad else None
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_bin_smoothed(ctx, J.ctypes.data_as(dp), dJ.ctypes.data_as(dp) if grad else None,
                                       C.c_void_p(stream)))
    return J[:n].reshape(shape), (dJ[:, :n].reshape((3,) + tuple(shape)) if grad else None)


def fte_grad(ctx, dL_dJ, stream: int):
    g = np.ascontiguousarray(dL_dJ, dtype=np.float64).ravel()
    out = np.zeros(3)
    dp = C.POINTER(C.c_double)
    _check(ctx, lib().fte_grad(ctx, g.ctypes.data_as(dp), out.ctypes.data_as(dp), C.c_void_p(stream)))
    return out


def fte_read_tangents(ctx, cap: int, stream: int):
    t = np.zeros((max(cap, 1), TANGENT_COLS))
    n = C.c_uint64()
    _check(ctx, lib().fte_read_tangents(ctx, t.ctypes.data_as(C.POINTER(C.c_double)), int(cap), C.byref(n),
                                        C.c_void_p(stream)))
    return t[: n.value]


def fte_save_state(ctx, stream: int) -> bytes:
    n = C.c_uint64()
    _check(ctx, lib().fte_state_size(ctx, C.byref(n), C.c_void_p(stream)))
    buf = C.create_string_buffer(n.value)
    _check(ctx, lib().fte_save_state(ctx, buf, n.value, C.c_void_p(stream)))
    return buf.raw


def fte_load_state(ctx, blob: bytes, stream: int):
    buf = C.create_string_buffer(bytes(blob), len(blob))
    _check(ctx, lib().fte_load_state(ctx, buf, len(blob), C.c_void_p(stream)))


def fte_autotune(ctx, trial_steps: int, stream: int):
    best = (C.c_int * 3)()
    _check(ctx, lib().fte_autotune(ctx, int(trial_steps), best, C.c_void_p(stream)))
    return tuple(best)


def fte_set_launch(ctx, block: int, steps_per_launch: int, compact_every: int, spatial_sort: int = 2):
    _check(ctx, lib().fte_set_launch(ctx, int(block), int(steps_per_launch), int(compact_every), int(spatial_sort)))


def fte_set_record_tile(ctx, tile_bytes: int):
    _check(ctx, lib().fte_set_record_tile(ctx, int(tile_bytes)))


def fte_set_lds_histogram(ctx, hist_bytes: int):
    _check(ctx, lib().fte_set_lds_histogram(ctx, int(hist_bytes)))


def fte_capture_begin(ctx, stream: int):
    _check(ctx, lib().fte_capture_begin(ctx, C.c_void_p(stream)))


def fte_capture_end(ctx, stream: int):
    g = C.c_void_p()
    _check(ctx, lib().fte_capture_end(ctx, C.c_void_p(stream), C.byref(g)))
    return g


def fte_graph_launch(ctx, graph, stream: int):
    _check(ctx, lib().fte_graph_launch(ctx, graph, C.c_void_p(stream)))


def fte_graph_destroy(graph):
    lib().fte_graph_destroy(graph)


def fte_reset(ctx, stream: int):
    _check(ctx, lib().fte_reset(ctx, C.c_void_p(stream)))


def fte_set_timing(ctx, enable: bool):
    _check(ctx, lib().fte_set_timing(ctx, int(bool(enable))))


# ----------------------------------------------------------------------------
# convenience: a context with torch-owned device buffers
# ----------------------------------------------------------------------------
class Simulation:
    """One context plus its device buffers (torch uint8 tensors on ``device``)."""

    def __init__(self, params: dict, grid: dict, n_max: int, device="cuda:0"):
        import torch
        self.torch = torch
        self.params = params
        self.grid = grid
        self.n_max = int(n_max)
        self.device = torch.device(device)
        self.sizes = fte_query_sizes(params, grid, n_max)
        s = self.sizes

        def buf(nbytes):
            return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=self.device)

        self.t_grid = buf(s.grid_bytes)
        self.t_index = buf(s.index_bytes)
        self.t_state_a = buf(s.state_bytes)
        self.t_state_b = buf(s.state_bytes)
        self.t_hist = buf(s.hist_bytes)
        self.t_work = buf(s.work_bytes)
        self.grad = bool(int(params.get("grad", 0)))
        self.t_tan_a = buf(s.tangent_bytes) if self.grad else None
        self.t_tan_b = buf(s.tangent_bytes) if self.grad else None
        self.bufs = fte_buffers(self.t_grid.data_ptr(), self.t_index.data_ptr(), self.t_state_a.data_ptr(),
                                self.t_state_b.data_ptr(), self.t_hist.data_ptr(), self.t_work.data_ptr(),
                                self.t_tan_a.data_ptr() if self.grad else None,
                                self.t_tan_b.data_ptr() if self.grad else None)
        self.ctx = fte_create(params)
        fte_bind_buffers(self.ctx, grid, n_max, self.bufs)
        self.n_runs = len(params.get("runs") or [])
        self.n_bins = (obs_bins(params), int(params.get("n_e", 1)), int(params.get("n_t", 1)))
        if self.n_runs:
            self.n_bins = (self.n_runs,) + self.n_bins

    @property
    def stream(self) -> int:
        return self.torch.cuda.current_stream(self.device).cuda_stream

    def load_grid(self, vb_sph):
        """vb_sph: float64 array [n_snap][n_leaves][cells][6] (numpy or torch)."""
        t = self.torch
        g = self.grid
        bx = g["bx"]
        want = (int(g["n_snap"]), len(g["leaves"]), bx[0] * bx[1] * bx[2], 6)
        if tuple(vb_sph.shape) != want:
            raise ValueError(f"wind data shape {tuple(vb_sph.shape)} != {want}")
        if isinstance(vb_sph, np.ndarray):
            vb = t.from_numpy(np.ascontiguousarray(vb_sph, dtype=np.float64)).to(self.device)
        else:
            vb = vb_sph.to(device=self.device, dtype=t.float64).contiguous()
        fte_load_grid(self.ctx, vb.data_ptr(), self.stream)
        del vb

    def plan_snapshot(self, k: int, sources, wind_speed_max: float):
        """With a leaf pool (grid n_pool > 0): choose the leaves snapshot k's
        slot holds; returns (input leaf ids, (gather, held, input) counts)."""
        return fte_plan_snapshot(self.ctx, k, sources, wind_speed_max, len(self.grid["leaves"]), self.stream)

    def load_snapshot(self, k: int, vb_all):
        """Derive snapshot k of a streaming grid into its slot from vb_all, a
        device float64 tensor [n_snap][n_leaves][cells][6] (only snapshots
        k-2 .. k+2 are read)."""
        t = self.torch
        if not (isinstance(vb_all, t.Tensor) and vb_all.is_cuda and vb_all.dtype == t.float64
                and vb_all.is_contiguous()):
            raise ValueError("vb_all must be a contiguous float64 CUDA tensor")
        ns = vb_all.shape[0]
        step = vb_all[0].numel() * 8
        base = vb_all.data_ptr()
        ptrs = [base + j * step if 0 <= j < ns else 0 for j in range(k - 2, k + 3)]
        fte_load_snapshot(self.ctx, k, ptrs, self.stream)

    def set_launch(self, block=256, steps_per_launch=64, compact_every=64, spatial_sort=1):
        fte_set_launch(self.ctx, block, steps_per_launch, compact_every, spatial_sort)

    def set_record_tile(self, tile_bytes):
        fte_set_record_tile(self.ctx, tile_bytes)

    def reset(self):
        fte_reset(self.ctx, self.stream)

    def set_timing(self, enable=True):
        fte_set_timing(self.ctx, enable)

    def set_lds_histogram(self, hist_bytes):
        fte_set_lds_histogram(self.ctx, hist_bytes)

    def capture_begin(self):
        """Record the following inject/step calls into a launch graph (nothing runs)."""
        fte_capture_begin(self.ctx, self.stream)

    def capture_end(self):
        """End the recording: a Graph to launch with graph_launch."""
        return Graph(fte_capture_end(self.ctx, self.stream))

    def graph_launch(self, graph):
        fte_graph_launch(self.ctx, graph.handle, self.stream)

    def inject(self, inj: dict, n: int, first_pid: int):
        fte_inject(self.ctx, inj, n, first_pid, self.stream)

    def step(self, n_steps: int):
        fte_step_n(self.ctx, n_steps, self.stream)

    def bin_observers(self, reset=False):
        return fte_bin_observers(self.ctx, self.n_bins, reset, self.stream)

    def bin_steady(self):
        """Time-integrated intensities [observer bin][E] (per run for an
        ensemble): the steady state of a Green's-function run."""
        shp = self.n_bins[:-1]
        return fte_bin_steady(self.ctx, shp, self.stream)

    def read_hist(self):
        n = int(np.prod(self.n_bins)) * int(self.params.get("n_batch", 32))
        return fte_read_hist(self.ctx, n, self.stream, self.n_runs)

    def autotune(self, trial_steps: int):
        """Try block sizes x compaction intervals from the current state (which
        is restored afterwards) and keep the fastest; returns (block,
        steps_per_launch, compact_every)."""
        return fte_autotune(self.ctx, trial_steps, self.stream)

    def bin_smoothed(self):
        """Smoothed intensities J[o][e][t] and (gradient mode) dJ[3][o][e][t]."""
        return fte_bin_smoothed(self.ctx, self.n_bins, self.grad, self.stream)

    def grad_of(self, dL_dJ):
        """Gradient of a loss with respect to (lambda_ref, kperp_ratio, gamma_inj)."""
        return fte_grad(self.ctx, dL_dJ, self.stream)

    def tangents(self):
        return fte_read_tangents(self.ctx, self.n_max, self.stream)

    def save_state(self) -> bytes:
        return fte_save_state(self.ctx, self.stream)

    def load_state(self, blob: bytes):
        fte_load_state(self.ctx, blob, self.stream)

    def stats(self) -> fte_stats:
        return fte_get_stats(self.ctx, self.stream)

    def particles(self) -> dict:
        return fte_read_particles(self.ctx, self.n_max, self.stream)

    def records(self):
        """Grid records as a tensor view [n_snap or slots][n_leaves][pcells][stride]."""
        t = self.torch
        bx = self.grid["bx"]
        pc = (bx[0] + 2) * (bx[1] + 2) * (bx[2] + 2)
        pp = make_params(self.params)
        dt = t.float64 if pp.precision == FTE_FP64 else t.float32
        rs = RECORD_STRIDE_KPERP if (pp.kperp_ratio > 0 or pp.lambda_perp > 0) else RECORD_STRIDE
        nl = len(self.grid["leaves"])
        ns = int(self.grid["n_snap"])
        slots = int(self.grid.get("n_slots", 0))
        ns = slots if 0 < slots < ns else ns       # a streaming grid holds its slots
        return self.t_grid.view(dt)[: ns * nl * pc * rs].view(ns, nl, pc, rs)

    def close(self):
        if getattr(self, "ctx", None):
            fte_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# differentiable smoothed intensities (torch.autograd)
# ----------------------------------------------------------------------------
def run_gradient(params: dict, grid: dict, vb_sph, injection: dict, n_particles: int, n_steps: int,
                 first_pid: int = 0, launch=None) -> "Simulation":
    """A gradient-mode Simulation after injecting ``n_particles`` and taking
    ``n_steps`` global steps; params must hold "smoothing" and grad=1."""
    sim = Simulation(dict(params, grad=1), grid, n_particles)
    sim.load_grid(vb_sph)
    if launch:
        sim.set_launch(*launch)
    sim.inject(injection, n_particles, first_pid)
    sim.step(n_steps)
    return sim


_Fn = None


def _function():
    global _Fn
    if _Fn is None:
        import torch

        class SmoothedIntensity(torch.autograd.Function):
            """J(theta) for theta = (lambda_ref, kperp_ratio, gamma_inj): the
            forward pass runs the workload in gradient mode and returns the
            smoothed intensities; the backward pass contracts the incoming
            dL/dJ on the device (fte_grad)."""

            @staticmethod
            def forward(ctx, theta, params, grid, vb_sph, injection, n_particles, n_steps, first_pid, launch):
                lam, kr, gam = (float(v) for v in theta.detach().cpu().tolist())
                p = dict(params, lambda_ref=lam, kperp_ratio=kr)
                inj = dict(injection, gamma_inj=gam)
                sim = run_gradient(p, grid, vb_sph, inj, n_particles, n_steps, first_pid, launch)
                J, _ = sim.bin_smoothed()
                ctx.sim = sim
                return torch.as_tensor(J, dtype=theta.dtype, device=theta.device)

            @staticmethod
            def backward(ctx, gJ):
                sim = ctx.sim
                g = sim.grad_of(gJ.detach().cpu().numpy())
                sim.close()
                ctx.sim = None
                return (torch.as_tensor(g, dtype=gJ.dtype, device=gJ.device),) + (None,) * 8

        _Fn = SmoothedIntensity
    return _Fn


def smoothed_intensity(theta, params: dict, grid: dict, vb_sph, injection: dict, n_particles: int, n_steps: int,
                       first_pid: int = 0, launch=None):
    """Differentiable J[o][e][t] as a function of the tensor theta =
    (lambda_ref, kperp_ratio, gamma_inj); backward gives dL/dtheta."""
    return _function().apply(theta, params, grid, vb_sph, injection, n_particles, n_steps, first_pid, launch)
