"""Closed-form checks of the HIP path itself (not through the oracle): in a
spherical grid holding a uniform field B along z and no flow, the SDE of
section 2.1 reduces to streaming along z and pitch-angle scattering, whose
moments are known exactly: the pitch-angle correlation <mu(t) mu(0)> =
<mu0^2> e^{-2 D t} for D_mumu = D (1 - mu^2), the finite-time parallel
displacement 2 kappa [t - (1 - e^{-2Dt})/(2D)] with kappa = v lambda / 3, the
long-time kappa_par = v lambda / 3 for Eq. 5, and the cross-field spread
4 kappa_perp t."""
import math

import numpy as np
import pytest

import fte_workloads as W

pytestmark = pytest.mark.gpu

AU = W.AU
DEG = W.DEG
E100 = 100 * W.KEV
EPS100 = E100 / (W.M_P * W.C_LIGHT ** 2)
P100 = math.sqrt(EPS100 * (EPS100 + 2))
V100 = W.C_LIGHT * P100 / math.sqrt(1 + P100 ** 2)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def F(torch_cuda):
    from paper_2404_12164_amd import fte
    fte.lib()
    return fte


def _uniform_z_grid():
    """0.9-1.1 au x colatitude 80-100 deg x longitude -10..10 deg, B = 5 nT
    along z in spherical components, V = 0."""
    n1, bx = (32, 64, 64), (8, 16, 16)
    g = W.grid_desc(0, 0.9 * AU, 0.2 * AU / 32, 80 * DEG, 20 * DEG / 64, -10 * DEG, 20 * DEG / 64, n1, bx,
                    W.uniform_leaves(n1, bx), 1, n_snap=1, phi_periodic=False)

    def wind(r, th, ph, t):
        z = np.zeros_like(r)
        return np.stack([z, z, z, 5e-9 * np.cos(th), -5e-9 * np.sin(th), z], axis=-1)

    return g, W.make_raw(g, wind)


def _run(F, torch, model, lam, kperp, n, steps, dt=1.0, snap_at=(), grad=None, eps=0.048):
    """FP64 run from one point with isotropic mu; particle states (and, with
    grad = dict of extra parameters, tangents) at t = 0, the snap_at steps and
    the end."""
    g, raw = _uniform_z_grid()
    p = dict(mass=W.M_P, dmm_model=model, dmm_norm=0, lambda_ref=lam, q=5 / 3, eps=eps, mu_floor=1e-4,
             kperp_ratio=kperp, dt=dt, r_in=0.5 * AU, r_out=2 * AU, seed=7, run_id=0, precision="fp64",
             observers=[], n_batch=1)
    if grad is not None:
        # gradient mode needs the smoothed sums; the tests read only the
        # tangents, so the one observer sits beyond the grid (no particle comes
        # within the kernels' reach, and no step contends for its sums)
        T = steps * dt
        p.update(observers=[(1.6 * AU, 90 * DEG, 0.0, 0.05 * AU, 10 * DEG, 10 * DEG)], e_min=50 * W.KEV,
                 dlne=math.log(4.0), n_e=1, t_ref=0.0, dT=2 * T, n_t=1, grad=1,
                 smoothing=dict(sigma_x=0.05 * AU, sigma_lne=0.5, sigma_t=T / 6), **grad)
    inj = dict(r=AU, th_lo=90 * DEG, th_hi=90 * DEG, ph_lo=0.0, ph_hi=0.0, e_lo=E100, e_hi=E100,
               gamma_inj=1.0, w0=1.0, pid0=0, n_total=n, k0=0, n_inj_steps=0)
    sim = F.Simulation(p, g, n)
    sim.load_grid(raw)
    sim.set_launch(256, 50, 0, 0)
    sim.inject(inj, n, 0)
    out = [sim.particles()]
    if grad is not None:
        out[0]["tan"] = sim.tangents()
    done = 0
    for s in list(snap_at) + [steps]:
        sim.step(s - done)
        done = s
        out.append(sim.particles())
        if grad is not None:
            out[-1]["tan"] = sim.tangents()
    torch.cuda.synchronize()
    sim.close()
    for o in out:
        assert np.all(o["status"] == 0)
        assert np.array_equal(o["pid"], out[0]["pid"])
    return out


def test_pitch_angle_correlation_iso(F, torch_cuda):
    Dc = 1e-3
    lam = V100 / (2 * Dc)                 # ISO: D = v / (2 lambda)
    N = 40000
    out = _run(F, torch_cuda, "iso", lam, 0.0, N, 1500, snap_at=(500, 1000))
    mu0 = out[0]["mu"]
    for t, o in zip((500, 1000, 1500), out[1:]):
        c = mu0 * o["mu"]
        want = np.mean(mu0 * mu0) * math.exp(-2 * Dc * t)
        assert abs(c.mean() - want) < 4 * c.std() / math.sqrt(N), (t, c.mean(), want)


def test_parallel_displacement_iso_finite_time(F, torch_cuda):
    Dc = 1e-3
    lam = V100 / (2 * Dc)
    kap = V100 * lam / 3
    N = 40000
    out = _run(F, torch_cuda, "iso", lam, 0.0, N, 3000, snap_at=(1000, 2000))
    z0 = out[0]["x"][:, 2]
    for t, o in zip((1000, 2000, 3000), out[1:]):
        dz2 = (o["x"][:, 2] - z0) ** 2
        want = 2 * kap * (t - (1 - math.exp(-2 * Dc * t)) / (2 * Dc))
        assert abs(dz2.mean() - want) < 4 * dz2.std() / math.sqrt(N) + 6 * Dc * want, (t, dz2.mean(), want)
        # no cross-field motion without kappa_perp (the field lines are straight)
        dxy = np.hypot(o["x"][:, 0] - out[0]["x"][:, 0], o["x"][:, 1] - out[0]["x"][:, 1])
        assert dxy.max() < 1e-3 * math.sqrt(want)      # only the interpolated b wobbles


def _eq5_integral(eps):
    """Int_{-1}^{1} (1 - mu^2) / (|mu| / (1 + |mu|) + eps) dmu by quadrature."""
    from scipy.integrate import quad
    return 2 * quad(lambda m: (1 - m * m) / (m / (1 + m) + eps), 0, 1, epsabs=0, epsrel=1e-12)[0]


def test_kappa_par_eq5_and_kappa_perp(F, torch_cuda):
    """Eq. 5 scattering from an isotropic start (mu stationary from t = 0):
    the displacement along B has <z^2>(t) = 2 kappa_par t - K + (terms that
    decay with the pitch-angle relaxation), so the slope between two late
    times is 2 kappa_par, kappa_par = v lambda / 3 for the MFP normalisation
    of D_mumu; across B the spread is 4 kappa_perp t."""
    lam = 3e8
    A = 3 * V100 * _eq5_integral(0.048) / (8 * lam)      # D_mumu = A (1 - mu^2)(|mu|/(1+|mu|) + eps)
    dt = 1.5e-3 / A
    ratio = 0.05
    N = 100000
    n1, n2 = 10000, 40000                                 # A t = 15 and 60
    out = _run(F, torch_cuda, "eq5", lam, ratio, N, n2, dt=dt, snap_at=(n1,))
    z0 = out[0]["x"][:, 2]
    q = (out[2]["x"][:, 2] - z0) ** 2 - (out[1]["x"][:, 2] - z0) ** 2
    scale = 2 * (n2 - n1) * dt * (V100 * lam / 3)
    k = q.mean() / scale
    s = q.std() / math.sqrt(N) / scale
    assert abs(k - 1) < 4 * s + 0.02, (k, s)
    dxy2 = (out[2]["x"][:, 0] - out[0]["x"][:, 0]) ** 2 + (out[2]["x"][:, 1] - out[0]["x"][:, 1]) ** 2
    want = 4 * ratio * V100 * lam / 3 * n2 * dt
    assert abs(dxy2.mean() - want) < 4 * dxy2.std() / math.sqrt(N), (dxy2.mean(), want)


_GRAD_RUNS = {}        # (model, eps, kink_sigma, A dt) -> estimate, shared by the cases


@pytest.mark.parametrize("model,eps,kink,adt", [("iso", 0.0, 0.0, 1.5e-3), ("eq5", 1.0, 0.03, 1.5e-3),
                                                ("eq5", 1.0, -1.0, 1.5e-3), ("eq5", 0.3, -1.0, 1.5e-3),
                                                ("eq5", 0.048, -1.0, 1e-4)])
def test_kappa_par_gradient(F, torch_cuda, model, eps, kink, adt):
    """The tangents against d kappa_par / d lambda = v / 3: the slope of
    <z^2> between late times is 2 kappa_par, so the slope of
    d<z^2>/d lambda = 2 <z dz/dlambda> is 2 v / 3.  For Eq. 5 this needs the
    Dirac term of d2D/dmu2 at mu = 0 (kink_sigma): the derivative of each
    sampled step alone recovers about 60% of it at eps = 1.  (At the paper's
    eps = 0.048 the tangent's multiplicative noise near mu = 0, of relative
    size sqrt(A dt / (2 eps)) per step, makes the Gaussian stand-in of the
    Dirac either biased, width 0.03, or heavy-tailed, narrower; eps = 1 pins
    the term itself.)  kink_sigma < 0 weights the Dirac by the bridge
    occupation of mu = 0 over each step instead, with no width to choose.
    At the paper's eps = 0.048 the bridge is pinned with steps that resolve
    the mu = 0 diffusion scale (A dt = 1e-4: one step's spread at mu = 0 is
    0.07 eps), between A t = 15 and 40."""
    lam = 3e8
    I = _eq5_integral(eps) if model == "eq5" else 4.0 / 3.0
    A = 3 * V100 * I / (8 * lam)
    dt = adt / A
    if adt >= 1e-3:
        N = 100000
        n1, n2 = 10000, 40000                             # A t = 15 and 60
    else:
        N = 40000
        n1, n2 = int(round(15 / adt)), int(round(40 / adt))
    res = {}
    for ks in sorted({0.0, kink}):
        if (model, eps, ks, adt) in _GRAD_RUNS:
            res[ks] = _GRAD_RUNS[(model, eps, ks, adt)]
            continue
        out = _run(F, torch_cuda, model, lam, 0.0, N, n2, dt=dt, snap_at=(n1,), grad=dict(kink_sigma=ks),
                   eps=eps if model == "eq5" else 0.048)
        z0 = out[0]["x"][:, 2]
        za, zb = out[1]["x"][:, 2] - z0, out[2]["x"][:, 2] - z0
        ta, tb = out[1]["tan"][:, 2], out[2]["tan"][:, 2]  # d z / d lambda_ref
        q = 2 * (zb * tb - za * ta)
        scale = 2 * (n2 - n1) * dt * (V100 / 3)
        res[ks] = _GRAD_RUNS[(model, eps, ks, adt)] = (q.mean() / scale, q.std() / math.sqrt(N) / scale)
        print(model, "eps", eps, "kink_sigma", ks, "d kappa / d lambda over v/3:", res[ks])
    k, s_ = res[kink]
    assert abs(k - 1) < 4 * s_ + 0.04, (k, s_)
    if kink != 0:
        k0, s0 = res[0.0]
        assert k0 < 0.8, (k0, s0)          # without the term the estimate falls well short


@pytest.mark.parametrize("rr,lo,hi", [(3.0, 4.35, 5.0), (2.0, 5.6, 6.8)])
def test_shock_acceleration_index(F, torch_cuda, rr, lo, hi):
    """First-order Fermi acceleration at a parallel shock on the GPU path: a
    radial wind jumping from U1 to U1/rr over a width 0.02 kappa/U1 at 20 au
    (where the shell is planar on the diffusion scale kappa/U2 = 0.13 au and
    the radial field's focusing length r/2 is 75 times larger), protons of
    v = 20 U1 injected at the shock with kappa independent of p.  The
    time-integrated spectrum just downstream follows f ~ p^-q with
    q = 3 rr / (rr - 1), 4.5 for rr = 3 and 6 for rr = 2 (the oracle's own pin
    measures ~4.7 and ~6.2 at v = 20 U1: the focused-transport spectrum is
    steeper by O(U1/v), so the bars are those of the oracle's pin).  The
    observer sums w v dt per ln E bin, so for E ~ p^2 they grow as p^(4 - q)."""
    torch = torch_cuda
    U1 = 4e5
    U2 = U1 / rr
    v0 = 20 * U1
    P0 = v0 / W.C_LIGHT / math.sqrt(1 - (v0 / W.C_LIGHT) ** 2)
    lam = 1e9
    kap = v0 * lam / 3
    w = 0.02 * kap / U1
    dt = min(0.04 * lam / v0, w / (3 * v0))
    tacc = 18 * kap / U1 ** 2
    n_steps = int(6 * tacc / dt)
    L = kap / U2
    r_s = 20 * AU
    up, down = 0.3 * AU, 1.0 * AU
    dxi = w / 4
    n_r = int(math.ceil((up + down) / dxi / 16)) * 16
    d = 1e-3
    n1, bx = (n_r, 4, 4), (16, 4, 4)
    g = W.grid_desc(0, r_s - up, dxi, 90 * DEG - 2 * d, d, 0.0, d, n1, bx, W.uniform_leaves(n1, bx), 1,
                    n_snap=1, phi_periodic=False)

    def wind(r, th, ph, t):
        z = r * 0.0
        V = U1 + (U2 - U1) * 0.5 * (1.0 + np.tanh((r - r_s) / w))
        return np.stack([V, z, z, 5e-9 * (r_s / r) ** 2, z, z], axis=-1)

    raw = W.make_raw(g, wind)
    E0 = W.M_P * W.C_LIGHT ** 2 * (math.sqrt(1 + P0 * P0) - 1)
    n_e = 40
    p = dict(mass=W.M_P, dmm_model="iso", dmm_norm=0, lambda_ref=lam, alpha=-1.0, p_ref=P0, kperp_ratio=0.0,
             dt=dt, r_in=r_s - up, r_out=r_s + down, seed=11, run_id=0, precision="mixed",
             observers=[(r_s + 5 * w + 0.5 * L, 90 * DEG, 2 * d, L, 4 * d, 4 * d)],
             e_min=E0, dlne=2 * math.log(4) / n_e, n_e=n_e, t_ref=0.0, dT=(n_steps + 10) * dt, n_t=1, n_batch=8)
    N = 200000
    inj = dict(r=r_s, th_lo=90 * DEG, th_hi=90 * DEG, ph_lo=2 * d, ph_hi=2 * d, e_lo=E0, e_hi=E0, gamma_inj=1.0,
               w0=1.0, pid0=0, n_total=N, k0=0, n_inj_steps=0)
    sim = F.Simulation(p, g, N)
    sim.load_grid(raw)
    sim.inject(inj, N, 0)
    left = n_steps
    while left > 0:
        k = min(20000, left)
        sim.step(k)
        left -= k
    torch.cuda.synchronize()
    sums, _ = sim.read_hist()
    sim.close()
    H = sums.reshape(n_e, -1).sum(axis=1)
    lnp = 0.5 * (np.arange(n_e) + 0.5) * p["dlne"]      # ln(p / p0) at the bin centres, E ~ p^2
    m = (lnp > math.log(1.15)) & (lnp < math.log(2.0)) & (H > 0)
    assert m.sum() > 10
    slope = np.polyfit(lnp[m], np.log(H[m]), 1, w=np.sqrt(H[m] / H[m].max()))[0]
    q = 4.0 - slope
    print("shock compression", rr, "steps", n_steps, "index q", q)
    assert lo < q < hi, q


def test_focusing_invariant_converges(F, torch_cuda):
    """Scatter-free focusing in a radial field B ~ r^-2 with no flow conserves
    the magnetic moment, (1 - mu^2) r^2 along each trajectory (through the
    mirror points of the inward-moving particles).  The HIP path keeps it to
    the order of the Euler-Maruyama step: the drift falls by half when dt
    halves."""
    torch = torch_cuda
    # fine angular cells: the derived div b takes central differences of the
    # Cartesian b across cells, whose relative error is ~ (cell angle)^2 / 6
    # (2.5% in the phi part at 22.5 deg cells, 3e-5 here)
    n1, bx = (128, 16, 16), (16, 16, 16)
    g = W.grid_desc(1, 0.1 * AU, math.log(20.0) / 128, 80 * DEG, 20 * DEG / 16, 0.4, 0.2 / 16, n1, bx,
                    W.uniform_leaves(n1, bx), 1, n_snap=1, phi_periodic=False)

    def wind(r, th, ph, t):
        z = r * 0.0
        return np.stack([z, z, z, 5e-9 * (AU / r) ** 2, z, z], axis=-1)

    raw = W.make_raw(g, wind)
    N = 2000
    inj = dict(r=0.2 * AU, th_lo=90 * DEG, th_hi=90 * DEG, ph_lo=0.5, ph_hi=0.5, e_lo=E100, e_hi=E100,
               gamma_inj=1.0, w0=1.0, pid0=0, n_total=N, k0=0, n_inj_steps=0)
    drift = []
    for dt in (2.0, 1.0):
        p = dict(mass=W.M_P, dmm_model="iso", dmm_norm=0, lambda_ref=1e30, kperp_ratio=0.0, dt=dt,
                 r_in=0.1 * AU, r_out=2 * AU, seed=3, run_id=0, precision="fp64", observers=[], n_batch=1)
        sim = F.Simulation(p, g, N)
        sim.load_grid(raw)
        sim.inject(inj, N, 0)
        a = sim.particles()
        sim.step(int(round(20000 / dt)))
        b = sim.particles()
        torch.cuda.synchronize()
        sim.close()
        # inward particles with |mu0| > 0.87 mirror only below r_in and are
        # absorbed (and compacted away); the others are all still held
        pos = {int(q): i for i, q in enumerate(a["pid"])}
        keep = b["status"] == 0
        ia = np.array([pos[int(q)] for q in b["pid"][keep]])
        assert len(ia) > 0.85 * N
        inv0 = (1 - a["mu"][ia] ** 2) * np.sum(a["x"][ia] ** 2, axis=1)
        inv1 = (1 - b["mu"][keep] ** 2) * np.sum(b["x"][keep] ** 2, axis=1)
        assert np.linalg.norm(b["x"][keep], axis=1).max() > 0.6 * AU   # the outward particles went far
        drift.append(np.median(np.abs(inv1 / inv0 - 1)))
    print("median relative drift of (1 - mu^2) r^2 at dt = 2, 1 s:", drift)
    assert drift[1] < 2e-3
    assert 1.5 < drift[0] / drift[1] < 2.6, drift


def test_adiabatic_deceleration_radial_wind(F, torch_cuda):
    """Particles scattered to isotropy (lambda << r) in a constant-speed radial
    wind are carried out with it and lose momentum at the rate div V / 3 =
    2 V / (3 r): along the flow ln p + (2/3) ln r stays constant, to
    corrections of order kappa / (V r) (about 1% here)."""
    torch = torch_cuda
    n1, bx = (128, 16, 16), (16, 16, 16)
    g = W.grid_desc(1, 0.1 * AU, math.log(20.0) / 128, 80 * DEG, 20 * DEG / 16, 0.4, 0.2 / 16, n1, bx,
                    W.uniform_leaves(n1, bx), 1, n_snap=1, phi_periodic=False)
    V = 4e5

    def wind(r, th, ph, t):
        z = r * 0.0
        return np.stack([z + V, z, z, 5e-9 * (AU / r) ** 2, z, z], axis=-1)

    raw = W.make_raw(g, wind)
    N = 20000
    lam = 1e8
    dt = 0.5
    p = dict(mass=W.M_P, dmm_model="iso", dmm_norm=0, lambda_ref=lam, kperp_ratio=0.0, dt=dt,
             r_in=0.1 * AU, r_out=2 * AU, seed=5, run_id=0, precision="fp64", observers=[], n_batch=1)
    inj = dict(r=0.2 * AU, th_lo=90 * DEG, th_hi=90 * DEG, ph_lo=0.5, ph_hi=0.5, e_lo=E100, e_hi=E100,
               gamma_inj=1.0, w0=1.0, pid0=0, n_total=N, k0=0, n_inj_steps=0)
    sim = F.Simulation(p, g, N)
    sim.load_grid(raw)
    sim.inject(inj, N, 0)
    a = sim.particles()
    sim.step(int(2e5 / dt))
    b = sim.particles()
    torch.cuda.synchronize()
    sim.close()
    assert np.all(b["status"] == 0) and len(b["pid"]) == N
    oa, ob = np.argsort(a["pid"]), np.argsort(b["pid"])
    ra = np.linalg.norm(a["x"][oa], axis=1)
    rb = np.linalg.norm(b["x"][ob], axis=1)
    change = np.mean(np.log(rb / ra))
    resid = np.mean(b["lnp"][ob] - a["lnp"][oa] + (2.0 / 3.0) * np.log(rb / ra))
    print("mean ln(r/r0)", change, "mean of dln p + (2/3) dln r", resid)
    assert change > 0.9                                  # carried out by a factor > 2.5
    assert abs(resid) < 0.03 * (2.0 / 3.0) * change, (resid, change)
