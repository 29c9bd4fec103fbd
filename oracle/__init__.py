"""FP64 CPU oracle for the focused-transport pseudo-particle method.

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, plain reference the GPU
library is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product path never
does.  It is written in plain C (``fte_oracle.c``) and loaded here with ctypes.
It shares no code with the GPU library: both read the same plain-Python
workload descriptions (dicts and numpy arrays from ``fte_workloads``) and each
marshals them into its own structures.

Parity status of each function (see the tests under ``tests/test_oracle_*.py``):
  philox4x32/normals      pinned: round structure against numpy's Philox4x64-10,
                          4x32 against rocRAND's host-compiled engine, moments
  dmm / dmm_integral      pinned: numerical quadrature of the definition;
                          the rigidity scaling lambda_par = lambda_ref (P/P_ref)^alpha
                          of D_mumu and kappa_perp by the parallel and cross-field
                          spreads at two momenta (alpha = 1/3 and -1)
  grid lookups/derive     pinned: brute-force leaf search, affine-field
                          exactness, Parker closed forms (2nd-order convergence)
  run (SDE step)          pinned: pitch-angle relaxation, parallel/perpendicular
                          diffusion, focusing and flow invariants, adiabatic
                          cooling, shock-acceleration index
  inject / finalize       pinned: distribution tests, intensity normalisation
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess
import sys

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fte_oracle.c")
_LIB = os.path.join(_HERE, "liboracle_fte.so")

DMM = {"iso": 0, "eq5": 1, "power_q": 2}
BG = {"grid": 0, "uniform": 1, "par_flow": 2, "perp_flow": 3, "radial": 4}
STATUS = {"active": 0, "abs_in": 1, "abs_out": 2, "out_of_domain": 3, "numeric": 4}


def build(force: bool = False, native: bool = False, out: str = None) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math).

    ``native`` builds the timing copy instead: -O3 -march=native for the
    host it is compiled on (so it must be built on the machine that runs it),
    with floating-point contraction off so that its arithmetic is the same as
    the portable build's; ``out`` is its path."""
    lib = out or _LIB
    if native:
        flags = ["-O3", "-march=native", "-ffp-contract=off"]
    else:
        flags = ["-O2"]
    if force or native or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(_SRC):
        cmd = ["gcc"] + flags + ["-std=gnu11", "-fopenmp", "-fPIC", "-shared", "-fno-fast-math",
                                 "-o", lib + ".tmp", _SRC, "-lm"]
        subprocess.check_call(cmd)
        os.replace(lib + ".tmp", lib)
    return lib


class OrParams(C.Structure):
    _fields_ = [
        ("mass", C.c_double), ("dmm_model", C.c_int), ("dmm_norm", C.c_int),
        ("lambda_ref", C.c_double), ("p_ref", C.c_double), ("alpha", C.c_double),
        ("q", C.c_double), ("eps", C.c_double), ("mu_floor", C.c_double),
        ("kperp_ratio", C.c_double), ("lambda_perp", C.c_double),
        ("dt", C.c_double), ("t0", C.c_double), ("r_in", C.c_double), ("r_out", C.c_double),
        ("check_bounds", C.c_int), ("run_id", C.c_int), ("seed", C.c_uint64),
        ("n_obs", C.c_int), ("obs", (C.c_double * 6) * 8), ("obs_nphi", C.c_int * 8), ("obs_omega", C.c_double * 8),
        ("e_min", C.c_double), ("dlne", C.c_double), ("n_e", C.c_int),
        ("t_ref", C.c_double), ("dT", C.c_double), ("n_t", C.c_int), ("n_batch", C.c_int),
        ("bg_kind", C.c_int), ("bg", C.c_double * 16),
        ("smooth", C.c_int), ("sig_x", C.c_double), ("sig_lne", C.c_double), ("sig_t", C.c_double),
    ]


class OrGridDesc(C.Structure):
    _fields_ = [
        ("xi_map", C.c_int), ("r_lo", C.c_double), ("dxi", C.c_double),
        ("th_lo", C.c_double), ("dth", C.c_double), ("ph_lo", C.c_double), ("dph", C.c_double),
        ("phi_periodic", C.c_int), ("n1", C.c_int * 3), ("bx", C.c_int * 3),
        ("n_levels", C.c_int), ("n_leaves", C.c_int), ("leaves", C.POINTER(C.c_int32)),
        ("n_snap_total", C.c_int), ("snap0", C.c_int), ("n_snap_held", C.c_int),
        ("t_s0", C.c_double), ("dt_s", C.c_double), ("raw", C.POINTER(C.c_double)),
    ]


class OrInjection(C.Structure):
    _fields_ = [
        ("r", C.c_double), ("th_lo", C.c_double), ("th_hi", C.c_double),
        ("ph_lo", C.c_double), ("ph_hi", C.c_double), ("e_lo", C.c_double), ("e_hi", C.c_double),
        ("gamma_inj", C.c_double), ("w0", C.c_double), ("r_weight", C.c_int), ("r_ref", C.c_double),
        ("pid0", C.c_uint64), ("n_total", C.c_uint64), ("k0", C.c_uint32), ("n_inj_steps", C.c_uint32),
        ("region", C.c_int), ("r_hi", C.c_double), ("divv_max", C.c_double), ("max_tries", C.c_uint32),
    ]


_lib = None


def use_native_build(out: str) -> str:
    """Build the -O3 -march=native timing copy at ``out`` on this host and
    make every later call of this module use it (the CPU-baseline timing);
    returns its path."""
    global _lib
    path = build(native=True, out=out)
    _lib = None
    lib(path)
    return path


def lib(path: str = None):
    global _lib
    if _lib is None:
        if path is None:
            build()
        L = C.CDLL(path or _LIB)
        dp = C.POINTER(C.c_double)
        u32p = C.POINTER(C.c_uint32)
        u64p = C.POINTER(C.c_uint64)
        i32p = C.POINTER(C.c_int32)
        lp = C.POINTER(C.c_long)
        L.or_philox4x32_10.argtypes = [u32p, u32p, u32p]
        L.or_philox4x64_10.argtypes = [u64p, u64p, u64p]
        L.or_philox_words.argtypes = [C.c_uint64, C.c_int, C.c_uint64, C.c_uint64, C.c_int, u32p]
        L.or_normals.argtypes = [C.c_uint64, C.c_int, C.c_uint64, C.c_uint64, dp]
        L.or_dmm_integral.argtypes = [C.c_int, C.c_double, C.c_double]
        L.or_dmm_integral.restype = C.c_double
        L.or_dmm_public.argtypes = [C.POINTER(OrParams), C.c_double, C.c_double, dp]
        L.or_grid_create.argtypes = [C.POINTER(OrGridDesc)]
        L.or_grid_create.restype = C.c_void_p
        L.or_grid_destroy.argtypes = [C.c_void_p]
        L.or_find_leaf.argtypes = [C.c_void_p, dp, C.POINTER(C.c_int), lp]
        L.or_find_leaf.restype = C.c_int
        L.or_raw_virtual.argtypes = [C.c_void_p, C.c_int, C.c_int, lp, dp]
        L.or_derived_virtual.argtypes = [C.c_void_p, C.c_int, C.c_int, lp, dp]
        L.or_grid_fields.argtypes = [C.c_void_p, dp, C.c_double, dp]
        L.or_grid_fields.restype = C.c_int
        L.or_fields_public.argtypes = [C.POINTER(OrParams), C.c_void_p, dp, C.c_double, dp]
        L.or_fields_public.restype = C.c_int
        L.or_run.argtypes = [C.POINTER(OrParams), C.c_void_p, C.c_long, dp, dp, dp, dp, u64p, u32p,
                             i32p, C.c_uint64, C.c_uint32, dp, dp, C.c_int]
        L.or_run.restype = C.c_uint64
        L.or_inject.argtypes = [C.POINTER(OrParams), C.c_void_p, C.POINTER(OrInjection), C.c_long, C.c_uint64,
                                dp, dp, dp, dp, u64p, u32p, i32p]
        L.or_finalize.argtypes = [C.POINTER(OrParams), dp, C.c_double, dp, dp]
        L.or_finalize_steady.argtypes = [C.POINTER(OrParams), dp, C.c_double, dp, dp]
        L.or_obs_bins.argtypes = [C.POINTER(OrParams)]
        L.or_obs_bins.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ----------------------------------------------------------------------------
# marshalling of plain workload dicts
# ----------------------------------------------------------------------------
def make_params(p: dict) -> OrParams:
    o = OrParams()
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
    o.check_bounds = int(p.get("check_bounds", 1))
    o.run_id = int(p.get("run_id", 0))
    o.seed = int(p.get("seed", 0))
    obs = p.get("observers", [])
    o.n_obs = len(obs)
    for i, ob in enumerate(obs):
        for k in range(6):
            o.obs[i][k] = ob[k]
        o.obs_nphi[i] = int(ob[6]) if len(ob) > 6 else 1
        o.obs_omega[i] = float(ob[7]) if len(ob) > 7 else 0.0
    o.e_min = p.get("e_min", 1.0)
    o.dlne = p.get("dlne", 1.0)
    o.n_e = int(p.get("n_e", 1))
    o.t_ref = p.get("t_ref", 0.0)
    o.dT = p.get("dT", 1.0)
    o.n_t = int(p.get("n_t", 1))
    o.n_batch = int(p.get("n_batch", 32))
    bk = p.get("bg_kind", "grid")
    o.bg_kind = BG[bk] if isinstance(bk, str) else int(bk)
    for i, v in enumerate(p.get("bg", [])):
        o.bg[i] = v
    sm = p.get("smoothing")
    if sm:
        o.smooth = 1
        o.sig_x, o.sig_lne, o.sig_t = sm["sigma_x"], sm["sigma_lne"], sm["sigma_t"]
    return o


def obs_bins(p: dict) -> int:
    """Observer bins: each observer (r, theta, phi, dr, dtheta, dphi[, n_phi[,
    omega]]) covers n_phi longitude bins."""
    return sum(int(ob[6]) if len(ob) > 6 and int(ob[6]) > 1 else 1 for ob in p.get("observers", []))


def hist_size(p: dict) -> int:
    return obs_bins(p) * int(p.get("n_e", 1)) * int(p.get("n_t", 1)) * int(p.get("n_batch", 32))


class Grid:
    """A block-AMR spherical grid held by the oracle.

    ``g`` is the plain grid description (``fte_workloads``), ``raw`` the
    snapshot data [held snapshots][leaf][cell][6] (V_r, V_th, V_ph, B_r, B_th,
    B_ph at cell centres, cells ordered xi fastest then theta then phi), and
    ``snap0`` the index of its first snapshot within the run.
    """

    def __init__(self, g: dict, raw: np.ndarray, snap0: int = 0):
        self.g = g
        self.raw = np.ascontiguousarray(raw, dtype=np.float64)
        self.leaves = np.ascontiguousarray(g["leaves"], dtype=np.int32)
        d = OrGridDesc()
        d.xi_map = int(g["xi_map"])
        d.r_lo = g["r_lo"]
        d.dxi = g["dxi"]
        d.th_lo = g["th_lo"]
        d.dth = g["dth"]
        d.ph_lo = g["ph_lo"]
        d.dph = g["dph"]
        d.phi_periodic = int(g["phi_periodic"])
        for a in range(3):
            d.n1[a] = int(g["n1"][a])
            d.bx[a] = int(g["bx"][a])
        d.n_levels = int(g["n_levels"])
        d.n_leaves = int(self.leaves.shape[0])
        d.leaves = _ptr(self.leaves, C.c_int32)
        d.n_snap_total = int(g["n_snap"])
        d.snap0 = int(snap0)
        d.n_snap_held = int(self.raw.shape[0])
        d.t_s0 = g.get("t_s0", 0.0)
        d.dt_s = g.get("dt_s", 1.0)
        d.raw = _ptr(self.raw, C.c_double)
        self._desc = d
        self.h = lib().or_grid_create(C.byref(d))

    def __del__(self):
        try:
            if getattr(self, "h", None):
                lib().or_grid_destroy(self.h)
                self.h = None
        except Exception:
            pass

    def find_leaf(self, s):
        s = np.ascontiguousarray(s, dtype=np.float64)
        lev = C.c_int()
        cell = np.zeros(3, dtype=np.int64)
        leaf = lib().or_find_leaf(self.h, _ptr(s, C.c_double), C.byref(lev), _ptr(cell, C.c_long))
        return leaf, lev.value, cell

    def raw_virtual(self, snap, L, c):
        c = np.ascontiguousarray(c, dtype=np.int64)
        out = np.zeros(6)
        lib().or_raw_virtual(self.h, snap, L, _ptr(c, C.c_long), _ptr(out, C.c_double))
        return out

    def derived_virtual(self, snap, L, c):
        c = np.ascontiguousarray(c, dtype=np.int64)
        out = np.zeros(13)
        lib().or_derived_virtual(self.h, snap, L, _ptr(c, C.c_long), _ptr(out, C.c_double))
        return out

    def fields(self, x, t):
        x = np.ascontiguousarray(x, dtype=np.float64)
        out = np.zeros(16)
        st = lib().or_grid_fields(self.h, _ptr(x, C.c_double), t, _ptr(out, C.c_double))
        return st, out[:13]


def philox4x32(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_ptr(c, C.c_uint32), _ptr(k, C.c_uint32), _ptr(out, C.c_uint32))
    return out


def philox4x64(ctr, key):
    c = np.ascontiguousarray(ctr, dtype=np.uint64)
    k = np.ascontiguousarray(key, dtype=np.uint64)
    out = np.zeros(4, dtype=np.uint64)
    lib().or_philox4x64_10(_ptr(c, C.c_uint64), _ptr(k, C.c_uint64), _ptr(out, C.c_uint64))
    return out


def philox_words(seed, run_id, n, pid, tag):
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox_words(seed, run_id, n, pid, tag, _ptr(out, C.c_uint32))
    return out


def normals(seed, run_id, n, pid):
    out = np.zeros(4)
    lib().or_normals(seed, run_id, n, pid, _ptr(out, C.c_double))
    return out


def dmm_integral(model, q=5.0 / 3.0, eps=0.0):
    m = DMM[model] if isinstance(model, str) else int(model)
    return lib().or_dmm_integral(m, q, eps)


def dmm(params: dict, P: float, mu: float):
    o = make_params(params)
    out = np.zeros(2)
    lib().or_dmm_public(C.byref(o), P, mu, _ptr(out, C.c_double))
    return out[0], out[1]


def fields(params: dict, grid, x, t):
    o = make_params(params)
    x = np.ascontiguousarray(x, dtype=np.float64)
    out = np.zeros(13)
    st = lib().or_fields_public(C.byref(o), grid.h if grid is not None else None,
                                _ptr(x, C.c_double), t, _ptr(out, C.c_double))
    return st, out


def make_injection(inj: dict) -> OrInjection:
    o = OrInjection()
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
    o.region = int(inj.get("region", 0))
    o.r_hi = inj.get("r_hi", inj["r"])
    o.divv_max = inj.get("divv_max", 0.0)
    o.max_tries = int(inj.get("max_tries", 4096))
    return o


class Particles:
    """Particle state arrays (FP64) in the oracle's own layout."""

    def __init__(self, n):
        self.x = np.zeros((n, 3))
        self.mu = np.zeros(n)
        self.lnp = np.zeros(n)
        self.w = np.zeros(n)
        self.pid = np.zeros(n, dtype=np.uint64)
        self.kinj = np.zeros(n, dtype=np.uint32)
        self.status = np.zeros(n, dtype=np.int32)

    def __len__(self):
        return self.mu.shape[0]

    def subset(self, idx):
        q = Particles(len(idx))
        for k in ("x", "mu", "lnp", "w", "pid", "kinj", "status"):
            setattr(q, k, np.ascontiguousarray(getattr(self, k)[idx]))
        return q

    def copy(self):
        return self.subset(np.arange(len(self)))


def inject(params: dict, inj: dict, n: int, first_pid: int, grid=None) -> Particles:
    """Particles of an injection; the region law (inj["region"] = 1) needs the
    grid it tests div V on."""
    o = make_params(params)
    io = make_injection(inj)
    if io.region and grid is None:
        raise ValueError("region injection needs the grid")
    p = Particles(n)
    lib().or_inject(C.byref(o), grid.h if grid is not None else None, C.byref(io), n, first_pid,
                    _ptr(p.x, C.c_double), _ptr(p.mu, C.c_double),
                    _ptr(p.lnp, C.c_double), _ptr(p.w, C.c_double), _ptr(p.pid, C.c_uint64),
                    _ptr(p.kinj, C.c_uint32), _ptr(p.status, C.c_int32))
    return p


def run(params: dict, grid, parts: Particles, n0: int, n_steps: int, hist=None, n_threads: int = 0,
        smooth=None) -> int:
    """Advance ``parts`` in place through steps n0..n0+n_steps-1; returns
    particle-steps taken.  ``hist`` (float64, ``hist_size(params)`` entries)
    is accumulated into when given; ``smooth`` (n_obs*n_e*n_t entries)
    receives the kernel-smoothed intensity sums when params has "smoothing"."""
    o = make_params(params)
    hp = _ptr(hist, C.c_double) if hist is not None else None
    sp = _ptr(smooth, C.c_double) if smooth is not None else None
    return lib().or_run(C.byref(o), grid.h if grid is not None else None, len(parts),
                        _ptr(parts.x, C.c_double), _ptr(parts.mu, C.c_double), _ptr(parts.lnp, C.c_double),
                        _ptr(parts.w, C.c_double), _ptr(parts.pid, C.c_uint64), _ptr(parts.kinj, C.c_uint32),
                        _ptr(parts.status, C.c_int32), n0, n_steps, hp, sp, n_threads)


def finalize(params: dict, hist: np.ndarray, w_inj: float):
    o = make_params(params)
    nob = obs_bins(params)
    n = nob * int(params["n_e"]) * int(params["n_t"])
    j = np.zeros(n)
    s = np.zeros(n)
    h = np.ascontiguousarray(hist, dtype=np.float64)
    lib().or_finalize(C.byref(o), _ptr(h, C.c_double), w_inj, _ptr(j, C.c_double), _ptr(s, C.c_double))
    shp = (nob, int(params["n_e"]), int(params["n_t"]))
    return j.reshape(shp), s.reshape(shp)


def finalize_steady(params: dict, hist: np.ndarray, w_inj: float):
    """Time-integrated intensities [observer bin][E] of a Green's-function
    run: the steady state for a unit injection rate (section 2.3)."""
    o = make_params(params)
    nob = obs_bins(params)
    n = nob * int(params["n_e"])
    j = np.zeros(n)
    s = np.zeros(n)
    h = np.ascontiguousarray(hist, dtype=np.float64)
    lib().or_finalize_steady(C.byref(o), _ptr(h, C.c_double), w_inj, _ptr(j, C.c_double), _ptr(s, C.c_double))
    return j.reshape(nob, int(params["n_e"])), s.reshape(nob, int(params["n_e"]))


def finalize_smoothed(params: dict, sm: np.ndarray, w_inj: float) -> np.ndarray:
    """Smoothed intensities J = sums / (4 pi W_inj), shaped (n_obs, n_e, n_t):
    the kernels already carry the 1/(dV dE dT) of the histogram estimator."""
    shp = (len(params["observers"]), int(params["n_e"]), int(params["n_t"]))
    return np.asarray(sm, dtype=np.float64).reshape(shp) / (4.0 * math.pi * w_inj)


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
