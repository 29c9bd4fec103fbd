"""The no-allocation variant of fte_bin_observers (finalize output staged in
the library's fixed device scratch) through the C ABI: the same intensities
and standard errors as fte_bin_observers, bit for bit, on two calls in a row
(the second on a context with fewer observer bins), and a clear error for a
context with more bins than the scratch holds."""
import math

import numpy as np
import pytest

import fte_workloads as W
from cases import near_observers

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


def _run(F, torch, params, n=2000, steps=1500):
    cfg = W.tiny_parker(n_particles=n)
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"])
    sim = F.Simulation(params, g, n)
    sim.load_grid(raw)
    sim.set_launch(256, 50, 100, 1)
    sim.inject(cfg["injection"], n, 0)
    sim.step(steps)
    torch.cuda.synchronize()
    return sim


def test_static_finalize_matches_bin_observers(F, torch_cuda):
    cfg = W.tiny_parker()
    big = near_observers(dict(cfg["params"], precision="mixed"))      # 3 observers x 10 x 84 bins
    small = dict(cfg["params"], precision="fp64", n_t=30)              # 1 observer x 10 x 30 bins
    for params in (big, small):
        sim = _run(F, torch_cuda, params)
        j0, s0 = sim.bin_observers()
        j1, s1 = F.fte_bin_observers_static(sim.ctx, sim.n_bins, False, sim.stream)
        assert j1.shape == j0.shape
        assert np.array_equal(j0, j1) and np.array_equal(s0, s1)
        assert (j0 > 0).sum() > 0 or params is small
        # reset clears the sums as fte_bin_observers does
        j2, _ = F.fte_bin_observers_static(sim.ctx, sim.n_bins, True, sim.stream)
        assert np.array_equal(j0, j2)
        j3, _ = sim.bin_observers()
        assert not j3.any()
        sim.close()
    # more bins than the scratch holds: refused, the context stays usable
    obs = [(0.5 * W.AU * (1 + 0.1 * k), 90 * W.DEG, 0.0, 0.05 * W.AU, 10 * W.DEG, 10 * W.DEG) for k in range(8)]
    huge = dict(cfg["params"], observers=obs, n_e=100, dlne=math.log(10) / 100, n_t=400, n_batch=4)
    assert 8 * 100 * 400 > 262144
    sim = _run(F, torch_cuda, huge, n=256, steps=20)
    with pytest.raises(F.FteError):
        F.fte_bin_observers_static(sim.ctx, sim.n_bins, False, sim.stream)
    j, _ = sim.bin_observers()
    assert j.shape == (8, 100, 400)
    sim.close()
