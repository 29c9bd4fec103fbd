"""Pins of the oracle's pieces of the paper's own workload (section 2.3):
ring observers that bin longitude and may corotate, the Green's-function to
steady-state time integral, and the injection law of Eq. 6 (uniform in volume
where the wind converges, weight r^-2)."""
import math

import numpy as np
import pytest

import fte_workloads as W

AU = W.AU
DEG = W.DEG
E100 = 100 * W.KEV
EPS100 = E100 / (W.M_P * W.C_LIGHT ** 2)
P100 = math.sqrt(EPS100 * (EPS100 + 2))
V100 = W.C_LIGHT * P100 / math.sqrt(1 + P100 ** 2)


def static(orc, n, x):
    p = orc.Particles(n)
    p.x[:] = x
    p.mu[:] = 0.0
    p.lnp[:] = math.log(P100)
    p.w[:] = 1.0
    p.pid[:] = np.arange(n, dtype=np.uint64)
    return p


def base(**kw):
    d = dict(mass=W.M_P, dmm_model="iso", lambda_ref=1e30, dt=10.0, bg_kind="uniform", bg=[0, 0, 0, 0, 0, 1],
             check_bounds=0, e_min=90 * W.KEV, dlne=math.log(110 / 90), n_e=1, t_ref=0.0, n_batch=4)
    d.update(kw)
    return d


def test_ring_observer_longitude_bins(orc):
    """One particle at rest at longitude 100 deg inside a ring of 12 bins of
    30 deg whose first bin is centred at 0: with no rotation every count
    lands in bin floor((100 + 15) / 30) = 3; rotating once through 360 deg
    over the run, the pattern sweeps every bin across the particle equally
    (to one step), and the particle moves to lower bin indices as time goes
    on (an eastward-moving pattern)."""
    phi_p = 100 * DEG
    x = (AU * math.cos(phi_p), AU * math.sin(phi_p), 0.0)
    N = 720
    ring = (AU, 90 * DEG, 0.0, 0.02 * AU, 4 * DEG, 30 * DEG, 12)
    par = base(observers=[ring + (0.0,)], dT=N * 10.0 + 1.0, n_t=1)
    h = np.zeros(orc.hist_size(par))
    orc.run(par, None, static(orc, 1, x), 0, N, h)
    per_bin = h.reshape(12, -1).sum(axis=1)
    assert per_bin[3] == pytest.approx(N * V100 * 10.0, rel=1e-12)
    assert np.count_nonzero(per_bin) == 1
    omega = 2 * math.pi / (N * 10.0)
    par = base(observers=[ring + (omega,)], dT=N * 10.0 / 24 + 1e-9, n_t=24)
    h = np.zeros(orc.hist_size(par))
    orc.run(par, None, static(orc, 1, x), 0, N, h)
    hb = h.reshape(12, 1, 24, -1).sum(axis=(1, 3))     # [ring bin][time bin of 15 deg of turn]
    steps = hb.sum(axis=1) / (V100 * 10.0)
    assert np.all(np.abs(steps - N / 12) <= 1.0 + 1e-9), steps
    dom = [int(np.argmax(hb[:, t])) for t in range(24)]
    seq = [d for i, d in enumerate(dom) if i == 0 or d != dom[i - 1]]
    # every ring bin once, in decreasing order (mod 12) from bin 3
    assert seq[0] == 3 and len(seq) == 12 and all((a - b) % 12 == 1 for a, b in zip(seq, seq[1:])), seq


def test_steady_state_time_integral(orc):
    """A uniform static population observed over T is a Green's function that
    stays constant for T; its time integral is j T with j = v n_E / (4 pi)
    (the normalisation of section 2.3), per unit injected weight."""
    N = 100000
    rng = np.random.default_rng(2)
    half = 0.1 * AU
    x = np.stack([AU + half * (2 * rng.random(N) - 1), half * (2 * rng.random(N) - 1),
                  half * (2 * rng.random(N) - 1)], axis=1)
    T = 30 * 10.0
    par = base(observers=[(AU, 90 * DEG, 0.0, 0.05 * AU, 4 * DEG, 4 * DEG)], dT=T / 3, n_t=3, n_batch=16)
    h = np.zeros(orc.hist_size(par))
    orc.run(par, None, static(orc, N, x), 0, 30, h)
    J, s = orc.finalize_steady(par, h, float(N))
    dE = 90 * W.KEV * (110 / 90 - 1)
    want = V100 / (4 * math.pi * (2 * half) ** 3 * dE) * T
    assert J[0, 0] == pytest.approx(want, rel=4 * s[0, 0] / want)
    assert s[0, 0] / want < 0.1
    # and it is the sum of the time-resolved intensities times dT
    j, _ = orc.finalize(par, h, float(N))
    assert J[0, 0] == pytest.approx(j[0, 0].sum() * T / 3, rel=1e-12)


def _converging_grid():
    """Uniform 1-level grid over 0.1-1.1 au, a radial wind whose speed falls
    as r^-3 inside r_b = 0.6 au (r^2 V decreasing: div V < 0) and as r^-1
    outside (div V > 0)."""
    n1, bx = (40, 8, 16), (8, 8, 8)
    g = W.grid_desc(0, 0.1 * AU, 1.0 * AU / 40, 70 * DEG, 40 * DEG / 8, 0.0, 2 * math.pi / 16, n1, bx,
                    W.uniform_leaves(n1, bx), 1, n_snap=1)
    r_b = 0.6 * AU

    def wind(r, th, ph, t):
        V = np.where(r < r_b, 4e5 * (r_b / r) ** 3, 4e5 * (r_b / r))
        z = np.zeros_like(r)
        return np.stack([V, z, z, 5e-9 * (AU / r) ** 2, z, z], axis=-1)

    return g, wind, r_b


def test_region_injection_law(orc):
    """Eq. 6: particles uniform in volume over the part of the shell sector
    where div V < 0, weight (r_ref/r)^2.  Every particle lies in a cell whose
    centre is inside r_b (the analytic sign change) or within one cell of it,
    the radii follow the uniform-in-volume law on [r_lo, r_b], angles are
    uniform in cos(theta) and phi, weights are exactly (r_ref/r)^2."""
    g, wind, r_b = _converging_grid()
    raw = W.make_raw(g, wind)
    G = orc.Grid(g, raw)
    par = base(observers=[], bg_kind="grid")
    inj = dict(r=0.2 * AU, r_hi=1.0 * AU, th_lo=85 * DEG, th_hi=95 * DEG, ph_lo=0.0, ph_hi=math.pi,
               e_lo=1e3 * W.KEV, e_hi=1e3 * W.KEV, gamma_inj=1.0, w0=1.0, r_weight=1, r_ref=AU, pid0=0,
               n_total=20000, region=1, divv_max=0.0, max_tries=4096)
    P = orc.inject(par, inj, 20000, 0, grid=G)
    assert np.all(P.status == 0)
    r = np.linalg.norm(P.x, axis=1)
    cell = g["dxi"]
    assert r.max() < r_b + cell and r.min() >= inj["r"]
    assert np.allclose(P.w, (AU / r) ** 2, rtol=1e-14)
    # uniform in volume on [r_lo, r_b - cell]: r^3 uniform
    sel = r < r_b - cell
    u = (r[sel] ** 3 - inj["r"] ** 3) / ((r_b - cell) ** 3 - inj["r"] ** 3)
    from scipy import stats
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    ct = P.x[:, 2] / r
    c1, c2 = math.cos(inj["th_lo"]), math.cos(inj["th_hi"])
    assert stats.kstest((ct - c1) / (c2 - c1), "uniform").pvalue > 1e-3
    ph = np.arctan2(P.x[:, 1], P.x[:, 0]) % (2 * math.pi)
    assert stats.kstest(ph / math.pi, "uniform").pvalue > 1e-3
    # an empty region gives up after max_tries and retires the particle
    none = orc.inject(par, dict(inj, r=0.7 * AU, r_hi=1.0 * AU, max_tries=64), 10, 0, grid=G)
    assert np.all(none.status == 4)
