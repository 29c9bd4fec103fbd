"""The paper's own workload pieces through the C ABI against the FP64 oracle:
the injection law of Eq. 6 (uniform in volume where the wind converges,
weight r^-2), ring observers that bin longitude and corotate, and the
Green's-function steady state (section 2.3)."""
import math

import numpy as np
import pytest

import fte_workloads as W
from cases import amr_cir_case

pytestmark = pytest.mark.gpu

AU = W.AU
DEG = W.DEG


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


def _case():
    p, g, inj = amr_cir_case()
    om = W.OMEGA_CIR
    p = dict(p, observers=[(0.9 * AU, 90 * DEG, 0.0, 0.1 * AU, 20 * DEG, 10 * DEG, 36, om),
                           (0.8 * AU, 90 * DEG, 0.0, 0.1 * AU, 30 * DEG, 20 * DEG, 18, 0.0),
                           (1.0 * AU, 90 * DEG, 200 * DEG, 0.1 * AU, 20 * DEG, 40 * DEG)],
             e_min=0.3 * 1e3 * W.KEV, dlne=math.log(10) / 8, n_e=8, n_t=9, dT=700.0)
    region = dict(inj, r=0.12 * AU, r_hi=1.1 * AU, th_lo=75 * DEG, th_hi=105 * DEG, ph_lo=0.0, ph_hi=2 * math.pi,
                  e_lo=1e3 * W.KEV, e_hi=1e3 * W.KEV, gamma_inj=1.0, w0=1.0, r_weight=1, r_ref=AU,
                  region=1, divv_max=0.0, max_tries=4096)
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    return p, g, region, raw


def test_region_injection_matches_oracle(F, torch_cuda, orc):
    """Same pids, same draws, same accepted points: positions, weights,
    first steps and statuses as the oracle's (the snapshot that decides
    div V < 0 changes during the stratified injection window)."""
    p, g, inj, raw = _case()
    G = orc.Grid(g, raw)
    sim = F.Simulation(p, g, 777)
    sim.load_grid(raw)
    sim.inject(inj, 400, 1000)
    sim.inject(inj, 377, 1400)
    got = sim.particles()
    sim.close()
    o = np.argsort(got["pid"])
    got = {k: v[o] for k, v in got.items()}
    ref = orc.inject(p, inj, 777, 1000, grid=G)
    assert np.array_equal(got["pid"], ref.pid)
    assert np.array_equal(got["kinj"], ref.kinj)
    assert np.array_equal(got["status"], ref.status)
    assert np.all(ref.status == 0)
    assert np.allclose(got["x"], ref.x, rtol=0, atol=1e-12 * AU)
    assert np.allclose(got["w"], ref.w, rtol=1e-12, atol=0)
    assert np.array_equal(got["mu"], ref.mu) and np.array_equal(got["lnp"], ref.lnp)
    # the law's support: each particle sits where the oracle's grid converges
    r = np.linalg.norm(ref.x, axis=1)
    assert r.min() >= inj["r"] and r.max() <= inj["r_hi"]
    assert len(np.unique(ref.kinj)) > 50


def test_rings_and_steady_state_match_oracle(F, torch_cuda, orc):
    """Region-injected 1 MeV protons over 300 steps: trajectories, the sums
    of a corotating 36-bin ring, a fixed 18-bin ring and a box observer, the
    binned intensities and the time-integrated (steady-state) intensities
    all as the oracle's."""
    p, g, inj, raw = _case()
    G = orc.Grid(g, raw)
    sim = F.Simulation(p, g, 777)
    sim.load_grid(raw)
    sim.set_launch(128, 25, 75, 2)
    sim.inject(inj, 777, 1000)
    sim.step(300)
    got = sim.particles()
    sums, w = sim.read_hist()
    jg, sg = sim.bin_observers()
    Jg, Sg = sim.bin_steady()
    sim.close()
    ref = orc.inject(p, inj, 777, 1000, grid=G)
    h = np.zeros(orc.hist_size(p))
    orc.run(p, G, ref, 0, 300, h)
    rp = {int(k): i for i, k in enumerate(ref.pid)}
    idx = np.array([rp[int(k)] for k in got["pid"]])
    live = got["status"] == 0
    assert np.array_equal(got["status"], ref.status[idx])
    dx = np.abs(got["x"][live] - ref.x[idx][live]).max()
    assert dx <= 1e-10 * AU, dx
    assert w == pytest.approx(ref.w.sum(), rel=1e-14)
    assert (h > 0).sum() > 40, "observers saw too little"
    assert h.reshape(36 + 18 + 1, -1).sum(axis=1)[:36].astype(bool).sum() > 3
    sc = np.abs(h).max()
    assert np.all(np.abs(sums - h) <= 1e-9 * np.maximum(np.abs(h), 1e-6 * sc))
    jo, so = orc.finalize(p, sums, w)
    assert np.allclose(jg, jo, rtol=1e-12, atol=0) and np.allclose(sg, so, rtol=1e-10, atol=1e-300)
    Jo, So = orc.finalize_steady(p, sums, w)
    assert Jg.shape == (55, 8)
    assert np.allclose(Jg, Jo, rtol=1e-12, atol=0) and np.allclose(Sg, So, rtol=1e-10, atol=1e-300)


def test_paper_workload_small_matches_oracle(F, torch_cuda, orc):
    """The paper's experiment end to end at reduced size (2 AMR levels, the
    corotating CIR with its frame flow, Eq. 5 with lambda ~ p^(1/3),
    lambda_perp, region injection, rings, steady state): FP64 trajectories
    and sums as the oracle's."""
    c = W.paper_cir(n_levels=2, n_particles=600, n_steps=1500, precision="fp64")
    g, p, inj = c["grid"], c["params"], c["injection"]
    raw = W.make_raw(g, c["wind"])
    sim = F.Simulation(p, g, 600)
    sim.load_grid(raw)
    sim.set_launch(256, 50, 150, 2)
    sim.inject(inj, 600, 0)
    sim.step(1500)
    got = sim.particles()
    sums, w = sim.read_hist()
    Jg, _ = sim.bin_steady()
    sim.close()
    G = orc.Grid(g, raw)
    ref = orc.inject(p, inj, 600, 0, grid=G)
    h = np.zeros(orc.hist_size(p))
    orc.run(p, G, ref, 0, 1500, h)
    rp = {int(k): i for i, k in enumerate(ref.pid)}
    idx = np.array([rp[int(k)] for k in got["pid"]])
    assert np.array_equal(got["status"], ref.status[idx])
    live = got["status"] == 0
    assert live.sum() > 300
    dx = np.abs(got["x"][live] - ref.x[idx][live]).max()
    assert dx <= 1e-10 * AU, dx
    assert (h > 0).sum() > 30
    sc = np.abs(h).max()
    assert np.all(np.abs(sums - h) <= 1e-9 * np.maximum(np.abs(h), 1e-6 * sc))
    Jo, _ = orc.finalize_steady(p, sums, w)
    assert np.allclose(Jg, Jo, rtol=1e-12, atol=0)


def test_sort_key_space_bounded_on_fine_grid(F, torch_cuda):
    """The paper's experiment on its 4-level grid (76,509 leaves) with 10^4
    particles: the spatial sort's key space is capped at 2^16 keys, so keys
    group pairs of consecutive leaves (more leaves than keys); trajectories
    are bit-identical to the ballot compaction's (storage order never changes
    a result)."""
    torch = torch_cuda
    c = W.paper_cir(n_levels=4, n_particles=10_000)
    g = c["grid"]
    assert len(g["leaves"]) > (1 << 16)
    raw = W.make_raw(g, c["wind"], xp=torch, device=torch.device("cuda:0"))
    outs = []
    for sort in (1, 0):
        sim = F.Simulation(c["params"], g, c["n_particles"])
        sim.load_grid(raw)
        sim.set_launch(256, 64, 64, sort)
        sim.inject(c["injection"], c["n_particles"], 0)
        sim.step(1280)
        torch.cuda.synchronize()
        outs.append((sim.particles(), sim.read_hist()[0], sim.stats()))
        sim.close()
    (a, sa, sta), (b, sb, stb) = outs
    oa, ob = np.argsort(a["pid"]), np.argsort(b["pid"])
    assert np.array_equal(a["pid"][oa], b["pid"][ob])
    for k in ("x", "mu", "lnp", "w", "status"):
        assert np.array_equal(a[k][oa], b[k][ob]), k
    assert sta.particle_steps == stb.particle_steps and sta.device_flags == 0
    assert np.allclose(sa, sb, rtol=1e-12, atol=1e-12 * max(np.abs(sa).max(), 1e-300))
