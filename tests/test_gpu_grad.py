"""Gradient mode of the HIP path (through the C ABI) against the FP64 oracle.

- Smoothed intensities J: the GPU's kernel-smoothed sums equal the oracle's on
  the same trajectories (FP64, 1e-9 relative).
- Tangents: every particle's pathwise derivative of (x, mu, ln p) with respect
  to lambda_ref and kperp_ratio against the oracle's central difference with
  common random numbers (same seed and pids, the parameter moved by 1e-5
  relative).
- dJ: the contracted gradient of several losses against the oracle's central
  difference of J with common random numbers at 1e-3 relative, within 5%
  (the acceptance bar of the differentiation workload).

The oracle needs no derivative code: the differences run it twice."""
import math

import numpy as np
import pytest

import fte_workloads as W
from cases import amr_cir_case

pytestmark = pytest.mark.gpu

AU = W.AU
DEG = W.DEG
N_STEPS = 300


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


def grad_case(precision="fp64"):
    """3-level AMR CIR case (Eq. 5, kappa_perp) with smoothing widths of
    0.04 au, 0.25 in ln E and 400 s at its three 0.3-au observers."""
    p, g, inj = amr_cir_case()
    p = dict(p, precision=precision, smoothing=dict(sigma_x=0.04 * AU, sigma_lne=0.25, sigma_t=400.0), grad=1)
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    injs = [(inj, 400, 1000), (inj, 377, 1400)]
    return p, g, inj, raw, injs


def gpu_grad_run(F, torch, p, g, raw, injs, n_steps, launch=(128, 25, 75, 2), chunks=None, tile=None):
    n_tot = sum(n for _, n, _ in injs)
    sim = F.Simulation(p, g, n_tot)
    sim.load_grid(raw)
    sim.set_launch(*launch)
    if tile is not None:
        sim.set_record_tile(tile)
    for inj, n, first in injs:
        sim.inject(inj, n, first)
    for c in chunks or [n_steps]:
        sim.step(c)
    torch.cuda.synchronize()
    out = dict(parts=sim.particles(), st=sim.stats())
    out["J"], out["dJ"] = sim.bin_smoothed()
    if p.get("grad"):
        out["tan"] = sim.tangents()
    out["sim"] = sim
    return out


def oracle_smoothed(orc, p, g, raw, injs, n_steps, G=None):
    G = G or orc.Grid(g, raw)
    parts = [orc.inject(p, inj, n, first) for inj, n, first in injs]
    P = parts[0]
    for q in parts[1:]:
        for k in ("x", "mu", "lnp", "w", "pid", "kinj", "status"):
            setattr(P, k, np.concatenate([getattr(P, k), getattr(q, k)]))
    w_inj = float(P.w.sum())
    n_obs = len(p["observers"])
    sm = np.zeros(n_obs * p["n_e"] * p["n_t"])
    orc.run(p, G, P, 0, n_steps, None, smooth=sm)
    return P, orc.finalize_smoothed(p, sm, w_inj)


def test_smoothed_intensity_fp64_parity(F, torch_cuda, orc):
    p, g, inj, raw, injs = grad_case()
    out = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS)
    out["sim"].close()
    _, J = oracle_smoothed(orc, p, g, raw, injs, N_STEPS)
    assert (J > 0).sum() > 30, "observers saw too little: the test would be vacuous"
    scale = J.max()
    assert np.all(np.abs(out["J"] - J) <= 1e-9 * np.maximum(np.abs(J), 1e-6 * scale)), \
        np.abs(out["J"] - J).max() / scale
    # the smoothing-only kernel (no tangents) accumulates the same sums
    p1 = dict(p, grad=0)
    out1 = gpu_grad_run(F, torch_cuda, p1, g, raw, injs, N_STEPS)
    out1["sim"].close()
    assert out1["dJ"] is None
    assert np.allclose(out1["J"], out["J"], rtol=1e-12, atol=1e-12 * scale)


def _fd_states(orc, p, g, raw, injs, key, h, G):
    """Oracle particles at parameter*(1 +- h)."""
    base = p[key]
    Pp, _ = oracle_smoothed(orc, dict(p, **{key: base * (1 + h)}), g, raw, injs, N_STEPS, G)
    Pm, _ = oracle_smoothed(orc, dict(p, **{key: base * (1 - h)}), g, raw, injs, N_STEPS, G)
    return Pp, Pm, 2 * h * base


def test_tangents_match_oracle_differences(F, torch_cuda, orc):
    """Per particle, d(x, y, z, mu, ln p)/d theta from the tangent kernel
    against (X(theta(1+h)) - X(theta(1-h))) / (2 h theta) of the oracle with
    the same noise, h = 1e-5.  The differences carry rounding noise of order
    1e-16 |X| / (h theta) - for the small pitch-angle and momentum derivatives
    the oracle's own differences at h = 1e-5 and 1e-6 already disagree by
    1e-5 (median) - and the map is piecewise smooth (trilinear cells, the |mu|
    kink of Eq. 5, reflections), so a particle whose two runs straddle a kink
    differs by up to the jump of one step's derivative.  The bar: median
    relative error below 1e-5 and below 1e-4 for at least 97% of particles."""
    p, g, inj, raw, injs = grad_case()
    out = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS)
    out["sim"].close()
    got, tan = out["parts"], out["tan"]
    G = orc.Grid(g, raw)
    for k, key in enumerate(("lambda_ref", "kperp_ratio")):
        Pp, Pm, den = _fd_states(orc, p, g, raw, injs, key, 1e-5, G)
        rp = {int(v): i for i, v in enumerate(Pp.pid)}
        idx = np.array([rp[int(v)] for v in got["pid"]])
        ok = (got["status"] == 0) & (Pp.status[idx] == 0) & (Pm.status[idx] == 0)
        assert ok.sum() > 300
        fd = np.concatenate([(Pp.x[idx] - Pm.x[idx]), (Pp.mu[idx] - Pm.mu[idx])[:, None],
                             (Pp.lnp[idx] - Pm.lnp[idx])[:, None]], axis=1)[ok] / den
        tg = tan[ok][:, 5 * k:5 * k + 5]
        scale = np.concatenate([np.full(3, np.median(np.abs(fd[:, :3]))), np.median(np.abs(fd[:, 3:]), axis=0)])
        assert np.all(scale > 0), scale
        rel = (np.abs(tg - fd) / (np.abs(fd) + 0.01 * scale)).max(axis=1)
        print(key, "particles", ok.sum(), "median rel", np.median(rel), "p97", np.quantile(rel, 0.97),
              "max", rel.max())
        assert np.quantile(rel, 0.97) < 1e-4, key
        assert np.median(rel) < 1e-5, key
    # d ln w / d gamma_inj = -ln(E0 / e_lo) of each particle's injected energy
    P0 = [orc.inject(p, i, n, f) for i, n, f in injs]
    lnp0 = {int(q): l for P in P0 for q, l in zip(P.pid, P.lnp)}
    P2 = np.exp(2 * np.array([lnp0[int(q)] for q in got["pid"]]))
    E0 = W.M_P * W.C_LIGHT ** 2 * P2 / (np.sqrt(1 + P2) + 1)
    dev = np.abs(tan[:, 10] + np.log(E0 / inj["e_lo"]))
    print("d ln w / d gamma deviation", dev.max())
    assert dev.max() < 1e-12


def _losses(shape, seed=7):
    rng = np.random.default_rng(seed)
    L = [np.ones(shape), rng.random(shape)]
    m = np.zeros(shape)
    m[0] = 1.0
    L.append(m)
    return L


def _fd_J(orc, p, g, raw, injs, h, G):
    """Central differences of the oracle's J for (lambda_ref, kperp_ratio,
    gamma_inj), common random numbers."""
    out = []
    for key in ("lambda_ref", "kperp_ratio"):
        base = p[key]
        _, Jp = oracle_smoothed(orc, dict(p, **{key: base * (1 + h)}), g, raw, injs, N_STEPS, G)
        _, Jm = oracle_smoothed(orc, dict(p, **{key: base * (1 - h)}), g, raw, injs, N_STEPS, G)
        out.append((Jp - Jm) / (2 * h * base))
    gam = injs[0][0]["gamma_inj"]
    inj_p = [(dict(i, gamma_inj=gam * (1 + h)), n, f) for i, n, f in injs]
    inj_m = [(dict(i, gamma_inj=gam * (1 - h)), n, f) for i, n, f in injs]
    _, Jp = oracle_smoothed(orc, p, g, raw, inj_p, N_STEPS, G)
    _, Jm = oracle_smoothed(orc, p, g, raw, inj_m, N_STEPS, G)
    out.append((Jp - Jm) / (2 * h * gam))
    return np.stack(out)


def test_gradient_matches_oracle_differences(F, torch_cuda, orc):
    """dL/d(lambda, kappa ratio, gamma) from the GPU against central
    differences (h = 1e-3, CRN) of the oracle's J, for three losses, within 5%."""
    p, g, inj, raw, injs = grad_case()
    out = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS)
    sim = out["sim"]
    G = orc.Grid(g, raw)
    fd = _fd_J(orc, p, g, raw, injs, 1e-3, G)
    dJ = out["dJ"]
    for wts in _losses(out["J"].shape):
        g_dev = sim.grad_of(wts)
        g_bin = np.array([(dJ[k] * wts).sum() for k in range(3)])
        g_fd = np.array([(fd[k] * wts).sum() for k in range(3)])
        print("grad", g_dev, "fd", g_fd)
        assert np.allclose(g_dev, g_bin, rtol=1e-10, atol=0)
        for k in range(3):
            assert abs(g_dev[k] - g_fd[k]) <= 0.05 * abs(g_fd[k]), (k, g_dev[k], g_fd[k])
    sim.close()


@pytest.mark.parametrize("precision,grad", [("fp64", 1), ("mixed", 1), ("mixed", 0)])
def test_gradient_launch_shape_invariance(F, torch_cuda, precision, grad):
    """Tangents and smoothed sums depend only on (pid, step): block size,
    launch length, compaction and the spatial sort move them with their
    particles.  On the mixed path every launch shape also moves each
    workgroup's LDS record tile (the tangent kernel's and, with grad = 0, the
    smoothed forward kernel's), so this also checks the tile paths against
    each other and against the tile switched off."""
    p, g, inj, raw, injs = grad_case(precision)
    p = dict(p, grad=grad)
    a = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS, launch=(256, 300, 0, 0))
    b = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS, launch=(64, 7, 21, 3), chunks=[13, 200, 87])
    runs = [a, b]
    if precision == "mixed":
        c = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS, launch=(128, 25, 75, 2), tile=0)
        runs.append(c)
    for r in runs:
        r["sim"].close()
    oa = np.argsort(a["parts"]["pid"])
    ma = a["parts"]["status"][oa] == 0
    for r in runs[1:]:
        ob = np.argsort(r["parts"]["pid"])
        mb = r["parts"]["status"][ob] == 0
        assert np.array_equal(a["parts"]["pid"][oa][ma], r["parts"]["pid"][ob][mb])
        for k in ("x", "mu", "lnp"):
            assert np.array_equal(a["parts"][k][oa][ma], r["parts"][k][ob][mb]), k
        if grad:
            assert np.array_equal(a["tan"][oa][ma], r["tan"][ob][mb])
        scale = np.abs(a["J"]).max()
        assert np.allclose(a["J"], r["J"], rtol=1e-11, atol=1e-12 * scale)
        if grad:
            scale = np.abs(a["dJ"]).max()
            assert np.allclose(a["dJ"], r["dJ"], rtol=1e-11, atol=1e-12 * scale)


@pytest.mark.parametrize("kink", [0.0, -1.0])
def test_mixed_precision_gradient(F, torch_cuda, kink):
    """The mixed path's gradient of the summed intensity against the FP64
    path's, same particles: within 5% (float step arithmetic moves each
    trajectory by rounding only); also with the bridge term of Eq. 5's
    mu = 0 kink, whose float and double evaluations differ in their erfcx."""
    p, g, inj, raw, injs = grad_case()
    p = dict(p, kink_sigma=kink)
    a = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS)
    b = gpu_grad_run(F, torch_cuda, dict(p, precision="mixed"), g, raw, injs, N_STEPS)
    for wts in _losses(a["J"].shape)[:2]:
        ga, gb = a["sim"].grad_of(wts), b["sim"].grad_of(wts)
        print("fp64", ga, "mixed", gb)
        assert np.all(np.abs(gb - ga) <= 0.05 * np.abs(ga)), (ga, gb)
    a["sim"].close()
    b["sim"].close()


def test_autograd_function(F, torch_cuda):
    """torch.autograd through the library: backward of sum(w * J) equals the
    device contraction of the same weights."""
    torch = torch_cuda
    p, g, inj, raw, injs = grad_case()
    theta = torch.tensor([p["lambda_ref"], p["kperp_ratio"], inj["gamma_inj"]], dtype=torch.float64,
                         requires_grad=True)
    inj1 = dict(inj, pid0=0, n_total=500)
    J = F.smoothed_intensity(theta, p, g, raw, inj1, 500, N_STEPS, first_pid=0)
    wts = torch.as_tensor(_losses(tuple(J.shape))[1])
    (J * wts).sum().backward()
    sim = F.run_gradient(p, g, raw, inj1, 500, N_STEPS)
    want = sim.grad_of(wts.numpy())
    J2, _ = sim.bin_smoothed()
    sim.close()
    assert np.allclose(J.detach().numpy(), J2, rtol=1e-12, atol=0)
    assert np.allclose(theta.grad.numpy(), want, rtol=1e-10, atol=0)


@pytest.mark.parametrize("kink", [0.03, -1.0])
def test_kink_term_moves_only_tangents(F, torch_cuda, kink):
    """kink_sigma adds Eq. 5's mu = 0 term to the tangents only (a Gaussian of
    that width, or, negative, the bridge occupation of mu = 0): positions and
    weights are bit-identical, J and the injection-index derivative equal to
    the rounding of their atomic sums, the lambda and kappa-ratio derivatives
    move."""
    p, g, inj, raw, injs = grad_case()
    a = gpu_grad_run(F, torch_cuda, p, g, raw, injs, N_STEPS)
    b = gpu_grad_run(F, torch_cuda, dict(p, kink_sigma=kink), g, raw, injs, N_STEPS)
    a["sim"].close()
    b["sim"].close()
    oa, ob = np.argsort(a["parts"]["pid"]), np.argsort(b["parts"]["pid"])
    for k in ("pid", "x", "mu", "lnp", "w", "status"):
        assert np.array_equal(a["parts"][k][oa], b["parts"][k][ob]), k
    sj = np.abs(a["J"]).max()
    assert np.allclose(a["J"], b["J"], rtol=1e-12, atol=1e-14 * sj)       # atomic summation order
    sg = np.abs(a["dJ"][2]).max()
    assert np.allclose(a["dJ"][2], b["dJ"][2], rtol=1e-11, atol=1e-13 * sg)
    assert np.array_equal(a["tan"][oa][:, 10], b["tan"][ob][:, 10])
    moved = np.abs(a["tan"][oa][:, :10] - b["tan"][ob][:, :10]).max(axis=1) > 0
    assert moved.sum() > 50
    assert not np.allclose(a["dJ"][:2], b["dJ"][:2], rtol=1e-6, atol=0)
