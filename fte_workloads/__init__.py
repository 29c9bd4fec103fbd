"""Seeded synthetic inputs for the focused-transport pseudo-particle path.

This module only *describes and generates inputs*: grid geometry and block-AMR
leaf lists, analytic solar-wind snapshots (V and B at cell centres), particle
sources, observers and run parameters, as plain dicts and arrays.  It holds none
of the transport method's arithmetic (no locate, interpolation, derivative, SDE
step, noise or binning).  Both the GPU library's binding and the CPU oracle
consume these descriptions, each through its own marshalling code.

The paper's own winds (Icarus/EUHFORIA snapshots driven by a synthetic tilted
slow-stream map, section 2.3) are not available, so analytic winds of the same
shape stand in for them: a steady Parker spiral and a corotating
interaction region (CIR) made of fast and slow streams with compressive ramps,
on the paper's domain (0.1-2 au, colatitude 30-150 deg, full longitude).
"""
from __future__ import annotations

import math

import numpy as np

AU = 1.495978707e11            # m
M_P = 1.67262192369e-27        # proton mass, kg
C_LIGHT = 299792458.0          # m/s
E_CHARGE = 1.602176634e-19     # C
KEV = 1e3 * E_CHARGE           # J
DEG = math.pi / 180.0
OMEGA_SYNODIC = 2.67e-6        # rad/s (section 2.3, region criterion)
OMEGA_CIR = 14.7 * DEG / 86400.0


# ----------------------------------------------------------------------------
# grid geometry and leaf lists
# ----------------------------------------------------------------------------
def uniform_leaves(n1, bx):
    """Level-1 leaves covering the whole domain, ordered I fastest."""
    nb = [n1[a] // bx[a] for a in range(3)]
    out = []
    for K in range(nb[2]):
        for J in range(nb[1]):
            for I in range(nb[0]):
                out.append((1, I, J, K))
    return np.array(out, dtype=np.int32)


def amr_leaves(n1, bx, n_levels, refine, phi_periodic=True):
    """Leaves of a block tree refined where ``refine(level, I, J, K)`` is True,
    then balanced so that blocks touching face-wise or diagonally differ by at
    most one level (the nesting rule of section 2.4).

    Returns an int32 array [n_leaves][4] = (level, I, J, K)."""
    nb1 = [n1[a] // bx[a] for a in range(3)]

    def nb(L):
        return [nb1[a] << (L - 1) for a in range(3)]

    refined = {L: set() for L in range(1, n_levels + 1)}
    # top-down refinement by the criterion
    exist = {1: {(I, J, K) for I in range(nb1[0]) for J in range(nb1[1]) for K in range(nb1[2])}}
    for L in range(1, n_levels):
        exist[L + 1] = set()
        for blk in exist[L]:
            if refine(L, *blk):
                refined[L].add(blk)
                I, J, K = blk
                for d in range(8):
                    exist[L + 1].add((2 * I + (d & 1), 2 * J + ((d >> 1) & 1), 2 * K + ((d >> 2) & 1)))

    def ancestor_leaf_level(L, blk):
        # level of the block that exists at or above (L, blk)
        I, J, K = blk
        M = L
        while M >= 1:
            if (I, J, K) in exist.get(M, set()):
                return M, (I, J, K)
            I, J, K = I >> 1, J >> 1, K >> 1
            M -= 1
        return None

    def add_refine(L, blk):
        refined[L].add(blk)
        I, J, K = blk
        exist.setdefault(L + 1, set())
        for d in range(8):
            exist[L + 1].add((2 * I + (d & 1), 2 * J + ((d >> 1) & 1), 2 * K + ((d >> 2) & 1)))

    changed = True
    while changed:
        changed = False
        for L in range(n_levels, 1, -1):
            for blk in list(exist.get(L, set())):
                if blk in refined.get(L, set()):
                    continue
                # a leaf at level L: every neighbour region must exist at level >= L-1
                I, J, K = blk
                n = nb(L)
                for dI in (-1, 0, 1):
                    for dJ in (-1, 0, 1):
                        for dK in (-1, 0, 1):
                            if dI == dJ == dK == 0:
                                continue
                            a, b, c = I + dI, J + dJ, K + dK
                            if a < 0 or a >= n[0] or b < 0 or b >= n[1]:
                                continue
                            if c < 0 or c >= n[2]:
                                if not phi_periodic:
                                    continue
                                c %= n[2]
                            # neighbour at level L-1 must exist (or be finer)
                            par = (a >> 1, b >> 1, c >> 1)
                            got = ancestor_leaf_level(L - 1, par)
                            if got is not None and got[0] < L - 1:
                                add_refine(got[0], got[1])
                                changed = True
    leaves = []
    for L in range(1, n_levels + 1):
        for blk in sorted(exist.get(L, set()), key=lambda b: (b[2], b[1], b[0])):
            if blk not in refined.get(L, set()):
                leaves.append((L,) + blk)
    return np.array(leaves, dtype=np.int32)


def grid_desc(xi_map, r_lo, dxi, th_lo, dth, ph_lo, dph, n1, bx, leaves, n_levels,
              n_snap=1, t_s0=0.0, dt_s=3600.0, phi_periodic=True):
    return dict(xi_map=int(xi_map), r_lo=float(r_lo), dxi=float(dxi), th_lo=float(th_lo), dth=float(dth),
                ph_lo=float(ph_lo), dph=float(dph), phi_periodic=int(phi_periodic), n1=list(n1), bx=list(bx),
                n_levels=int(n_levels), leaves=np.asarray(leaves, dtype=np.int32), n_snap=int(n_snap),
                t_s0=float(t_s0), dt_s=float(dt_s))


def cell_centres(g, xp=np, device=None):
    """Cell-centre (r, theta, phi) for every leaf cell, each [n_leaves, cells],
    cells ordered xi fastest, then theta, then phi.  ``xp`` is numpy or torch."""
    leaves = np.asarray(g["leaves"])
    bx = g["bx"]
    ii = np.arange(bx[0])
    jj = np.arange(bx[1])
    kk = np.arange(bx[2])
    K, J, I = np.meshgrid(kk, jj, ii, indexing="ij")
    I, J, K = I.ravel(), J.ravel(), K.ravel()      # xi fastest
    lev = leaves[:, 0:1].astype(np.float64)
    h = np.ldexp(1.0, (1 - leaves[:, 0:1]).astype(np.int64))
    cxi = leaves[:, 1:2] * bx[0] + I[None, :]
    cth = leaves[:, 2:3] * bx[1] + J[None, :]
    cph = leaves[:, 3:4] * bx[2] + K[None, :]
    del lev
    xi = (cxi + 0.5) * g["dxi"] * h
    r = g["r_lo"] * np.exp(xi) if g["xi_map"] == 1 else g["r_lo"] + xi
    th = g["th_lo"] + (cth + 0.5) * g["dth"] * h
    ph = g["ph_lo"] + (cph + 0.5) * g["dph"] * h
    if xp is np:
        return r, th, ph
    import torch
    return (torch.as_tensor(r, device=device), torch.as_tensor(th, device=device),
            torch.as_tensor(ph, device=device))


# ----------------------------------------------------------------------------
# analytic winds: return V_sph(3), B_sph(3) stacked on the last axis
# ----------------------------------------------------------------------------
def _xp(a):
    try:
        import torch
        if isinstance(a, torch.Tensor):
            return torch
    except ImportError:  # pragma: no cover
        pass
    return np


def parker_wind(r, th, ph, t, V0=400e3, B1au=5e-9, omega=OMEGA_SYNODIC, polarity=1.0):
    """Steady Parker spiral: radial V0, B_r ~ r^-2, B_phi = -B_r omega r sin(theta)/V0,
    with |B| = B1au at 1 au in the equator (outward polarity)."""
    xp = _xp(r)
    a1 = omega * AU / V0
    Br0 = B1au / math.sqrt(1.0 + a1 * a1)
    Br = polarity * Br0 * (AU / r) ** 2
    Bph = -Br * omega * r * xp.sin(th) / V0
    z = r * 0.0
    return xp.stack([z + V0, z, z, Br, z, Bph], -1)


def cir_wind(r, th, ph, t, Vs=330e3, Vf=650e3, omega=OMEGA_CIR, U=500e3, r_B=0.1 * AU,
             psi_R=60 * DEG, psi_F=75 * DEG, psi_S=250 * DEG, width=10 * DEG, width_rare=40 * DEG,
             B0=5e-9 * 100.0):
    """Corotating fast/slow stream pattern seen in the inertial frame.

    Source phase psi = phi - omega t + omega (r - r_B)/U (the spiral of the
    region criterion, section 2.3, Eq. 7).  Along psi the speed falls from the
    fast stream Vf to (Vs+Vf)/2 across the reverse ramp at psi_R and to Vs across
    the forward ramp at psi_F (both compressive), and rises back to Vf across a
    wide rarefaction ramp at psi_S.  Ramp widths narrow as r_B/r so the ramps
    steepen outward.  B is radial ~ r^-2 wound by the local speed."""
    xp = _xp(r)
    two_pi = 2.0 * math.pi
    psi = ph - omega * t + omega * (r - r_B) / U
    psi = psi - two_pi * xp.floor(psi / two_pi)
    w = width * (r_B / r)
    Vm = 0.5 * (Vs + Vf)

    def H(x):
        return 0.5 * (1.0 + xp.tanh(x))

    V = (Vf - (Vf - Vm) * H((psi - psi_R) / w) - (Vm - Vs) * H((psi - psi_F) / w)
         + (Vf - Vs) * H((psi - psi_S) / (width_rare * (r_B / r) ** 0.5)))
    Br = B0 * (r_B / r) ** 2
    Bph = -Br * omega * r * xp.sin(th) / V
    z = r * 0.0
    return xp.stack([V, z, z, Br, z, Bph], -1)


def cir_wind_corotating(r, th, ph, t, omega=OMEGA_CIR, **kw):
    """The CIR pattern of cir_wind frozen at t = 0 and seen in the frame
    corotating with it: the same radial speed and field, plus the frame's
    flow V_phi = -omega r sin(theta), which makes V parallel to B (no
    electric field in this frame), so the background is steady there."""
    xp = _xp(r)
    f = cir_wind(r, th, ph, 0.0 * t, omega=omega, **kw)
    vph = -omega * r * xp.sin(th)
    return xp.stack([f[..., 0], f[..., 1], vph, f[..., 3], f[..., 4], f[..., 5]], -1)


def cir_shocked_wind(r, th, ph, t, Vs=330e3, Vf=650e3, omega=OMEGA_CIR, U=500e3, r_B=0.1 * AU,
                     psi_R=60 * DEG, psi_F=75 * DEG, psi_S=250 * DEG, comp=3.0, width_shock=0.2 * DEG,
                     width_if=2.5 * DEG, width_rare=40 * DEG, B0=5e-9 * 100.0):
    """The CIR pattern of cir_wind with its two compressive ramps turned into
    shocks of compression ratio comp.

    The pattern is steady in the frame corotating with it, where its surfaces
    psi = const are spirals whose normal sees the flow component proportional
    to V_r - U.  Mass flux through a shock of compression comp divides that
    component by comp, so the fast wind Vf drops to U + (Vf - U)/comp across
    the reverse shock at psi_R, the slow wind Vs is reached from
    U - (U - Vs)/comp across the forward shock at psi_F, the two downstream
    speeds join across a stream interface midway (width width_if), and a wide
    rarefaction at psi_S returns to Vf.  The shock width (width_shock in psi)
    is far below a grid cell, so the grid holds each shock as a one-cell
    jump.  B is radial ~ r^-2, wound by the local speed."""
    xp = _xp(r)
    two_pi = 2.0 * math.pi
    psi = ph - omega * t + omega * (r - r_B) / U
    psi = psi - two_pi * xp.floor(psi / two_pi)
    v_r2 = U + (Vf - U) / comp
    v_f2 = U - (U - Vs) / comp

    def H(x):
        return 0.5 * (1.0 + xp.tanh(x))

    V = (Vf - (Vf - v_r2) * H((psi - psi_R) / width_shock)
         - (v_r2 - v_f2) * H((psi - 0.5 * (psi_R + psi_F)) / width_if)
         - (v_f2 - Vs) * H((psi - psi_F) / width_shock)
         + (Vf - Vs) * H((psi - psi_S) / (width_rare * (r_B / r) ** 0.5)))
    Br = B0 * (r_B / r) ** 2
    Bph = -Br * omega * r * xp.sin(th) / V
    z = r * 0.0
    return xp.stack([V, z, z, Br, z, Bph], -1)



def affine_fields(r_or_xi, th, ph, t, coef):
    """A field affine in (xi, theta, phi, t) for each of the six components;
    coef is [6][5] = constant, d/dxi, d/dtheta, d/dphi, d/dt."""
    xp = _xp(th)
    comps = [coef[k][0] + coef[k][1] * r_or_xi + coef[k][2] * th + coef[k][3] * ph + coef[k][4] * t
             for k in range(6)]
    return xp.stack(comps, -1)


def make_raw(g, wind, snaps=None, xp=np, device=None, dtype=None, **kw):
    """Snapshot data [snap][leaf][cell][6] for the given wind function."""
    r, th, ph = cell_centres(g, xp, device)
    snaps = range(g["n_snap"]) if snaps is None else snaps
    out = []
    for k in snaps:
        t = g["t_s0"] + k * g["dt_s"]
        out.append(wind(r, th, ph, t, **kw))
    if xp is np:
        return np.ascontiguousarray(np.stack(out, 0), dtype=np.float64)
    import torch
    res = torch.stack(out, 0).contiguous()
    return res.to(dtype) if dtype is not None else res


# ----------------------------------------------------------------------------
# workloads
# ----------------------------------------------------------------------------
def _bins(e_lo_kev, e_hi_kev, n_e):
    return dict(e_min=e_lo_kev * KEV, dlne=math.log(e_hi_kev / e_lo_kev) / n_e, n_e=n_e)


def tiny_parker(n_particles=2000, n_steps=5000, precision="fp64"):
    """Steady Parker wind on a uniform 64 x 32 x 64 spherical grid (0.1-2 au),
    2,000 monoenergetic 100 keV protons from a 10 x 10 deg patch at 0.1 au,
    power-law D_mumu (q = 5/3, lambda = 0.3 au), dt = 10 s, one observer at 1 au
    with 10 log energy bins 50-500 keV and 60 ten-minute time bins."""
    n1, bx = (64, 32, 64), (16, 16, 16)
    g = grid_desc(0, 0.1 * AU, 1.9 * AU / 64, 30 * DEG, 120 * DEG / 32, 0.0, 2 * math.pi / 64, n1, bx,
                  uniform_leaves(n1, bx), 1, n_snap=1)
    params = dict(mass=M_P, dmm_model="power_q", dmm_norm=0, lambda_ref=0.3 * AU, p_ref=1.0, alpha=0.0,
                  q=5.0 / 3.0, eps=0.0, mu_floor=1e-4, kperp_ratio=0.0, lambda_perp=0.0, dt=10.0, t0=0.0,
                  r_in=0.05 * AU, r_out=2.0 * AU, check_bounds=1, run_id=0, seed=0,
                  observers=[(1.0 * AU, 90 * DEG, 0.0, 0.05 * AU, 10 * DEG, 10 * DEG)],
                  t_ref=0.0, dT=600.0, n_t=60, n_batch=32, precision=precision, **_bins(50.0, 500.0, 10))
    # footpoint magnetically connected to the observer: dphi = omega (0.9 au) / V
    phc = OMEGA_SYNODIC * 0.9 * AU / 400e3
    inj = dict(r=0.1 * AU, th_lo=85 * DEG, th_hi=95 * DEG, ph_lo=phc - 5 * DEG, ph_hi=phc + 5 * DEG,
               e_lo=100 * KEV, e_hi=100 * KEV, gamma_inj=1.0, w0=1.0, pid0=0, n_total=n_particles,
               k0=0, n_inj_steps=0)
    return dict(name="tiny_parker", grid=g, wind=parker_wind, wind_kw={}, params=params, injection=inj,
                n_particles=n_particles, n_steps=n_steps)


def cir_grid(n_levels=2, n_snap=48, n_r=256, n_th=60, n_ph=192, bx=(16, 12, 16)):
    """Stretched CIR grid: r_i = 0.1 * 1.01^i au, colatitude 30-150 deg,
    full longitude, blocks refined once where the region criterion (section
    2.3, Eq. 7) puts the compression band during the run, near the equator."""
    n1 = (n_r, n_th, n_ph)
    dxi = math.log(1.01)
    dth = 120 * DEG / n_th
    dph = 2 * math.pi / n_ph
    r_B, U, om = 0.1 * AU, 500e3, OMEGA_CIR
    t_span = (n_snap - 1) * 3600.0
    lo, hi = 45 * DEG, 90 * DEG + om * t_span + 15 * DEG

    def refine(L, I, J, K):
        if L >= n_levels:
            return False
        h = 2.0 ** (1 - L)
        th0 = 30 * DEG + J * bx[1] * dth * h
        th1 = th0 + bx[1] * dth * h
        if th1 <= 55 * DEG or th0 >= 125 * DEG:
            return False
        r0 = 0.1 * AU * math.exp(I * bx[0] * dxi * h)
        r1 = 0.1 * AU * math.exp((I + 1) * bx[0] * dxi * h)
        p0 = K * bx[2] * dph * h
        p1 = p0 + bx[2] * dph * h
        # phi-hat = phi + (r - r_B) omega / U over the block
        a = p0 + (r0 - r_B) * om / U
        b = p1 + (r1 - r_B) * om / U
        two = 2 * math.pi
        for sh in (-two, 0.0, two):
            if a + sh < hi and b + sh > lo:
                return True
        return False

    leaves = amr_leaves(n1, bx, n_levels, refine) if n_levels > 1 else uniform_leaves(n1, bx)
    return grid_desc(1, 0.1 * AU, dxi, 30 * DEG, dth, 0.0, dph, n1, bx, leaves, n_levels,
                     n_snap=n_snap, t_s0=0.0, dt_s=3600.0)


def cir_time_dependent(n_particles=10_000_000, n_steps=16920, precision="mixed", n_levels=2, n_snap=48):
    """CIR wind, 48 hourly snapshots on a stretched 2-level grid, 10^7
    protons 5-50 keV with an E^-4 spectrum injected continuously at 0.1 au over
    47 h, lambda = 0.2 au, three observers at 1 au (phi = 0, 30, 60 deg)."""
    g = cir_grid(n_levels=n_levels, n_snap=n_snap)
    r_out = 0.1 * AU * math.exp(g["n1"][0] * g["dxi"])
    params = dict(mass=M_P, dmm_model="power_q", dmm_norm=0, lambda_ref=0.2 * AU, p_ref=1.0, alpha=0.0,
                  q=5.0 / 3.0, eps=0.0, mu_floor=1e-4, kperp_ratio=0.0, lambda_perp=0.0, dt=10.0, t0=0.0,
                  r_in=0.05 * AU, r_out=r_out, check_bounds=1, run_id=0, seed=0,
                  observers=[(1.0 * AU, 90 * DEG, p * DEG, 0.05 * AU, 10 * DEG, 10 * DEG) for p in (0, 30, 60)],
                  t_ref=0.0, dT=600.0, n_t=282, n_batch=32, precision=precision, **_bins(2.0, 100.0, 10))
    inj = dict(r=0.1 * AU, th_lo=30 * DEG, th_hi=150 * DEG, ph_lo=0.0, ph_hi=2 * math.pi,
               e_lo=5 * KEV, e_hi=50 * KEV, gamma_inj=4.0, w0=1.0, pid0=0, n_total=n_particles,
               k0=0, n_inj_steps=n_steps)
    return dict(name="cir_time_dependent", grid=g, wind=cir_wind, wind_kw={}, params=params, injection=inj,
                n_particles=n_particles, n_steps=n_steps)


def cir_differentiation(n_particles=1_000_000, n_steps=8000, precision="mixed", n_snap=48, kink_sigma=0.03):
    """Gradient workload: the CIR wind and grid of cir_time_dependent, 10^6
    protons (5-50 keV, E^-4) injected continuously over 8,000 steps of 10 s,
    Eq. 5 scattering with lambda = 0.2 au, kappa_perp / kappa_par = 0.02, and
    intensities at the three 1-au observers smoothed by Gaussians of 0.05 au,
    0.1 in ln E and 10 min; differentiated with respect to (lambda, kappa
    ratio, injection index), the mu = 0 term of Eq. 5 in the tangents carried
    by a Gaussian of width kink_sigma."""
    cfg = cir_time_dependent(n_particles=n_particles, n_steps=n_steps, precision=precision, n_snap=n_snap)
    params = dict(cfg["params"], dmm_model="eq5", eps=0.048, kperp_ratio=0.02,
                  n_t=int(math.ceil(n_steps * 10.0 / 600.0)),
                  smoothing=dict(sigma_x=0.05 * AU, sigma_lne=0.1, sigma_t=600.0), grad=1, kink_sigma=kink_sigma)
    return dict(cfg, name="cir_differentiation", params=params)


def cir_ensemble(n_runs=64, precision="mixed", seed=0, n_snap=57, particle_range=(1e4, 1e6),
                 step_range=(2000, 20000)):
    """Batched ensemble: n_runs independent runs on the CIR grid and wind (one
    refinement level), lambda log-uniform in [0.05, 1] au, kappa_perp/kappa_par
    uniform in [0, 0.05], particle counts log-uniform in particle_range, step
    counts uniform in step_range; each run injects its particles (5-50 keV,
    E^-4, r = 0.1 au) continuously over its own steps, pids in disjoint
    ranges.  57 hourly snapshots cover 20,000 steps of 10 s."""
    rng = np.random.default_rng(seed)
    g = cir_grid(n_levels=2, n_snap=n_snap)
    lam = np.exp(rng.uniform(math.log(0.05), math.log(1.0), n_runs)) * AU
    kr = rng.uniform(0.0, 0.05, n_runs)
    npart = np.exp(rng.uniform(math.log(particle_range[0]), math.log(particle_range[1]), n_runs)).astype(np.int64)
    nstep = rng.integers(step_range[0], step_range[1] + 1, n_runs)
    runs = [dict(lambda_ref=float(lam[r]), kperp_ratio=float(kr[r]), n_steps=int(nstep[r])) for r in range(n_runs)]
    r_out = 0.1 * AU * math.exp(g["n1"][0] * g["dxi"])
    params = dict(mass=M_P, dmm_model="power_q", dmm_norm=0, lambda_ref=0.2 * AU, p_ref=1.0, alpha=0.0,
                  q=5.0 / 3.0, eps=0.0, mu_floor=1e-4, kperp_ratio=0.0, lambda_perp=0.0, dt=10.0, t0=0.0,
                  r_in=0.05 * AU, r_out=r_out, check_bounds=1, run_id=0, seed=0,
                  observers=[(1.0 * AU, 90 * DEG, p * DEG, 0.05 * AU, 10 * DEG, 10 * DEG) for p in (0, 30, 60)],
                  t_ref=0.0, dT=600.0, n_t=int(math.ceil(step_range[1] * 10.0 / 600.0)), n_batch=8,
                  precision=precision, runs=runs, **_bins(2.0, 100.0, 10))
    injections = []
    pid = 0
    for r in range(n_runs):
        n = int(npart[r])
        injections.append(dict(r=0.1 * AU, th_lo=30 * DEG, th_hi=150 * DEG, ph_lo=0.0, ph_hi=2 * math.pi,
                               e_lo=5 * KEV, e_hi=50 * KEV, gamma_inj=4.0, w0=1.0, pid0=pid, n_total=n,
                               k0=0, n_inj_steps=int(nstep[r]), run=r))
        pid += n
    return dict(name="cir_ensemble", grid=g, wind=cir_wind, wind_kw={}, params=params, injections=injections,
                n_particles=int(npart.sum()), n_steps=int(nstep.max()), runs=runs)


def paper_cir(n_levels=2, n_particles=1_000_000, n_steps=36000, precision="mixed"):
    """The paper's own experiment (section 2.3) on the synthetic CIR: the
    pattern in its corotating frame (one steady snapshot) on a stretched grid
    r_i = 0.1 * 1.01^i au to 2.06 au with n_levels AMR levels on the band the
    region criterion (Eq. 7) selects; 1 MeV protons injected at t = 0
    (a Green's-function run) uniformly where div V < 0 within 0.12-2 au and
    colatitude 90 +- 2 deg, weight r^-2 (Eq. 6); Eq. 5 scattering
    (eps = 0.048) with lambda = 0.3 au at 1 MeV scaling as p^(1/3),
    lambda_perp = 3e-4 au; absorbing at 0.1 and 2 au; longitude rings of 2
    deg bins at 0.5, 1.0, 1.5 and 1.8 au in the equator, 12 log energy bins
    0.25-16 MeV; the steady state is the time integral (fte_bin_steady)."""
    g = cir_grid(n_levels=n_levels, n_snap=1, n_r=304)
    E1 = 1e3 * KEV
    eps1 = E1 / (M_P * C_LIGHT ** 2)
    p1 = math.sqrt(eps1 * (eps1 + 2.0))
    rings = [(rr * AU, 90 * DEG, 1 * DEG, 0.05 * AU, 4 * DEG, 2 * DEG, 180, 0.0) for rr in (0.5, 1.0, 1.5, 1.8)]
    params = dict(mass=M_P, dmm_model="eq5", dmm_norm=0, lambda_ref=0.3 * AU, p_ref=p1, alpha=1.0 / 3.0,
                  q=5.0 / 3.0, eps=0.048, mu_floor=1e-4, kperp_ratio=0.0, lambda_perp=3e-4 * AU, dt=10.0,
                  t0=0.0, r_in=0.1 * AU, r_out=2.0 * AU, check_bounds=1, run_id=0, seed=0, observers=rings,
                  t_ref=0.0, dT=n_steps * 10.0 + 10.0, n_t=1, n_batch=16, precision=precision,
                  **_bins(250.0, 16000.0, 12))
    inj = dict(r=0.12 * AU, r_hi=2.0 * AU, th_lo=88 * DEG, th_hi=92 * DEG, ph_lo=0.0, ph_hi=2 * math.pi,
               e_lo=E1, e_hi=E1, gamma_inj=1.0, w0=1.0, r_weight=1, r_ref=AU, pid0=0, n_total=n_particles,
               k0=0, n_inj_steps=0, region=1, divv_max=0.0, max_tries=65536)
    return dict(name="paper_cir", grid=g, wind=cir_wind_corotating, wind_kw={}, params=params, injection=inj,
                n_particles=n_particles, n_steps=n_steps, ring_radii_au=[0.5, 1.0, 1.5, 1.8])


def particle_spec_like(inj, **over):
    d = dict(inj)
    d.update(over)
    return d


def cir_largest_grid(n_snap=96):
    """Stretched 3-level grid for the shocked CIR: 128 log-spaced radial cells
    over 0.1-2 au (ratio 20^(1/128) per cell), 32 colatitude cells over 30-150
    deg (the block rule of three levels needs a multiple of 8 there; 30 would
    not divide), 96 longitude cells, blocks of 16 x 8 x 16 cells; level 2 on
    the band the compression region sweeps during the run (the region
    criterion of section 2.3, Eq. 7, for the pattern speed U) near the
    equator, level 3 on a narrower band around both shocks."""
    n1, bx = (128, 32, 96), (16, 8, 16)
    dxi = math.log(20.0) / n1[0]
    dth = 120 * DEG / n1[1]
    dph = 2 * math.pi / n1[2]
    r_B, U, om = 0.1 * AU, 500e3, OMEGA_CIR
    sweep = om * (n_snap - 1) * 3600.0
    bands = {1: (45 * DEG, 90 * DEG + sweep + 15 * DEG, 55 * DEG, 125 * DEG),
             2: (55 * DEG, 80 * DEG + sweep + 5 * DEG, 65 * DEG, 115 * DEG)}

    def refine(L, I, J, K):
        if L not in bands:
            return False
        lo, hi, t_lo, t_hi = bands[L]
        h = 2.0 ** (1 - L)
        th0 = 30 * DEG + J * bx[1] * dth * h
        th1 = th0 + bx[1] * dth * h
        if th1 <= t_lo or th0 >= t_hi:
            return False
        r0 = r_B * math.exp(I * bx[0] * dxi * h)
        r1 = r_B * math.exp((I + 1) * bx[0] * dxi * h)
        p0 = K * bx[2] * dph * h
        p1 = p0 + bx[2] * dph * h
        a = p0 + (r0 - r_B) * om / U
        b = p1 + (r1 - r_B) * om / U
        two = 2 * math.pi
        return any(a + sh < hi and b + sh > lo for sh in (-two, 0.0, two))

    leaves = amr_leaves(n1, bx, 3, refine)
    return grid_desc(1, r_B, dxi, 30 * DEG, dth, 0.0, dph, n1, bx, leaves, 3, n_snap=n_snap, t_s0=0.0,
                     dt_s=3600.0)


def cir_largest(n_particles=100_000_000, precision="mixed", n_snap=96):
    """Largest workload: the shocked CIR (compression 3 at both shocks) on the
    3-level grid of cir_largest_grid, 96 hourly snapshots; 10^8 protons of
    1-100 keV (E^-4) injected continuously at 0.1 au over the 95 h the
    snapshots span (34,200 steps of 10 s); power-law D_mumu with
    lambda = 0.2 au, kappa_perp / kappa_par = 0.01; five observers at 0.5,
    0.75, 1.0, 1.25 and 1.5 au on the equator at longitude 0, 20 log energy
    bins 1-100 keV x 288 time bins of 20 min."""
    g = cir_largest_grid(n_snap=n_snap)
    n_steps = int(round((n_snap - 1) * 3600.0 / 10.0))
    params = dict(mass=M_P, dmm_model="power_q", dmm_norm=0, lambda_ref=0.2 * AU, p_ref=1.0, alpha=0.0,
                  q=5.0 / 3.0, eps=0.0, mu_floor=1e-4, kperp_ratio=0.01, lambda_perp=0.0, dt=10.0, t0=0.0,
                  r_in=0.05 * AU, r_out=2.0 * AU, check_bounds=1, run_id=0, seed=0,
                  observers=[(r * AU, 90 * DEG, 0.0, 0.05 * AU, 10 * DEG, 10 * DEG)
                             for r in (0.5, 0.75, 1.0, 1.25, 1.5)],
                  t_ref=0.0, dT=1200.0, n_t=288, n_batch=32, precision=precision, **_bins(1.0, 100.0, 20))
    inj = dict(r=0.1 * AU, th_lo=30 * DEG, th_hi=150 * DEG, ph_lo=0.0, ph_hi=2 * math.pi,
               e_lo=1 * KEV, e_hi=100 * KEV, gamma_inj=4.0, w0=1.0, pid0=0, n_total=n_particles,
               k0=0, n_inj_steps=n_steps)
    return dict(name="cir_largest", grid=g, wind=cir_shocked_wind, wind_kw={}, params=params, injection=inj,
                n_particles=n_particles, n_steps=n_steps)
