"""The step kernel deals runs of consecutive particle slices to each XCD
(a permutation of the workgroups once a launch has more than 8 x 32 of them):
a launch with enough workgroups to be permuted gives the trajectories and
sums of one with too few to be (the same particles, 64- against 256-thread
workgroups), bit for bit, on both paths."""
import math

import numpy as np
import pytest

import fte_workloads as W

pytestmark = pytest.mark.gpu


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


def _run(F, torch, p, g, vb, inj, n, block, steps):
    sim = F.Simulation(p, g, n)
    sim.load_grid(vb)
    sim.set_launch(block, 64, 64, 1)
    sim.inject(inj, n, 0)
    sim.step(steps)
    torch.cuda.synchronize()
    out = sim.particles()
    sums, w = sim.read_hist()
    sim.close()
    m = out["status"] == 0
    o = np.argsort(out["pid"][m])
    return {k: out[k][m][o] for k in ("pid", "x", "mu", "lnp")}, sums, w


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_xcd_slice_order_matches_plain_order(F, torch_cuda, precision):
    torch = torch_cuda
    n = 40000                   # 625 workgroups of 64 (permuted), 157 of 256 (not)
    cfg = W.cir_time_dependent(n_particles=n, n_snap=4)
    g = cfg["grid"]
    obs = [(r * W.AU, 90 * W.DEG, 0.0, 0.05 * W.AU, 20 * W.DEG, 10 * W.DEG, 36) for r in (0.15, 0.25)]
    p = dict(cfg["params"], precision=precision, observers=obs, n_t=12)
    inj = dict(cfg["injection"], n_total=n, pid0=0, k0=0, n_inj_steps=0)
    vb = W.make_raw(g, cfg["wind"], xp=torch, device=torch.device("cuda:0"))
    steps = int(g["dt_s"] / p["dt"]) + 130
    a, sa, wa = _run(F, torch, p, g, vb, inj, n, 64, steps)
    b, sb, wb = _run(F, torch, p, g, vb, inj, n, 256, steps)
    assert len(a["pid"]) > n // 2
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    assert (sa > 0).sum() > 10
    assert wa == pytest.approx(wb, rel=1e-14)
    assert np.allclose(sa, sb, rtol=1e-12, atol=1e-14 * np.abs(sa).max())


def test_lds_histogram_matches_global_sums(F, torch_cuda):
    """The observer histogram accumulated in LDS per launch (the budget of
    fte_set_lds_histogram) against every contribution a global atomic: the
    same trajectories (the smaller record tile it leaves moves no value) and
    the same sums up to the order of the additions."""
    torch = torch_cuda
    n = 30000
    cfg = W.cir_time_dependent(n_particles=n, n_snap=4)
    g = cfg["grid"]
    # 2 rings x 18 bins x 10 energies x <= 3 time bins per launch x 2 batches
    # x 8 bytes = 17 KB: within the LDS budget below
    obs = [(r * W.AU, 90 * W.DEG, 0.0, 0.05 * W.AU, 20 * W.DEG, 20 * W.DEG, 18) for r in (0.15, 0.25)]
    p = dict(cfg["params"], precision="mixed", observers=obs, n_t=12, n_batch=2)
    inj = dict(cfg["injection"], n_total=n, pid0=0, k0=0, n_inj_steps=0)
    vb = W.make_raw(g, cfg["wind"], xp=torch, device=torch.device("cuda:0"))
    steps = int(g["dt_s"] / p["dt"]) + 130
    out = []
    for hist_bytes in (0, 32768):
        sim = F.Simulation(p, g, n)
        sim.load_grid(vb)
        sim.set_launch(256, 64, 64, 1)
        sim.set_lds_histogram(hist_bytes)
        sim.inject(inj, n, 0)
        sim.step(steps)
        torch.cuda.synchronize()
        parts = sim.particles()
        sums, w = sim.read_hist()
        sim.close()
        m = parts["status"] == 0
        o = np.argsort(parts["pid"][m])
        out.append(({k: parts[k][m][o] for k in ("pid", "x", "mu", "lnp")}, sums, w))
    (a, sa, wa), (b, sb, wb) = out
    for key in a:
        assert np.array_equal(a[key], b[key]), key
    assert (sa > 0).sum() > 10
    assert np.array_equal(sa > 0, sb > 0)
    assert np.allclose(sa, sb, rtol=1e-12, atol=1e-14 * np.abs(sa).max())
    with pytest.raises(F.FteError):
        s = F.Simulation(p, g, 10)
        try:
            s.set_lds_histogram(1 << 20)
        finally:
            s.close()
