"""Checkpoint / resume through the C ABI: a run saved part way and restored
into a fresh context continues exactly as the uninterrupted run (trajectories,
tangents, observer and smoothed sums), and mismatched or damaged blobs are
rejected."""
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
    p = dict(p, smoothing=dict(sigma_x=0.04 * AU, sigma_lne=0.25, sigma_t=400.0), grad=1)
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    return p, g, inj, raw


def _sim(F, p, g, raw, n):
    sim = F.Simulation(p, g, n)
    sim.load_grid(raw)
    sim.set_launch(128, 25, 75, 2)
    return sim


def _snapshot(sim):
    parts = sim.particles()
    o = np.argsort(parts["pid"])
    J, dJ = sim.bin_smoothed()
    sums, w = sim.read_hist()
    return dict(parts={k: v[o] for k, v in parts.items()}, tan=sim.tangents()[o], J=J, dJ=dJ, sums=sums, w=w,
                st=sim.stats())


def test_resume_matches_uninterrupted_run(F, torch_cuda):
    p, g, inj, raw = _case()
    a = _sim(F, p, g, raw, 777)
    a.inject(inj, 777, 1000)
    a.step(300)
    A = _snapshot(a)
    a.close()

    b = _sim(F, p, g, raw, 777)
    b.inject(inj, 777, 1000)
    b.step(120)
    blob = b.save_state()
    b.close()
    c = _sim(F, p, g, raw, 800)
    c.load_state(blob)
    assert c.stats().global_step == 120
    c.step(180)
    C = _snapshot(c)
    c.close()

    live_a = A["parts"]["status"] == 0
    live_c = C["parts"]["status"] == 0
    assert np.array_equal(A["parts"]["pid"][live_a], C["parts"]["pid"][live_c])
    for k in ("x", "mu", "lnp", "w", "kinj"):
        assert np.array_equal(A["parts"][k][live_a], C["parts"][k][live_c]), k
    assert np.array_equal(A["tan"][live_a], C["tan"][live_c])
    assert A["w"] == pytest.approx(C["w"], rel=1e-14)     # atomic sums: order-dependent rounding
    assert np.allclose(A["sums"], C["sums"], rtol=1e-12, atol=0)
    sJ = np.abs(A["J"]).max()
    assert np.allclose(A["J"], C["J"], rtol=1e-12, atol=1e-14 * sJ)
    sd = np.abs(A["dJ"]).max()
    assert np.allclose(A["dJ"], C["dJ"], rtol=1e-11, atol=1e-13 * sd)
    assert A["st"].particle_steps == C["st"].particle_steps
    assert list(A["st"].n_retired) == list(C["st"].n_retired)


def test_rejects_mismatched_or_damaged_state(F, torch_cuda):
    p, g, inj, raw = _case()
    a = _sim(F, p, g, raw, 777)
    a.inject(inj, 777, 1000)
    a.step(30)
    blob = a.save_state()
    a.close()
    other = _sim(F, dict(p, seed=p["seed"] + 1), g, raw, 777)
    with pytest.raises(F.FteError):
        other.load_state(blob)
    other.close()
    small = _sim(F, p, g, raw, 100)
    with pytest.raises(F.FteError):
        small.load_state(blob)            # more particles than the capacity
    small.close()
    same = _sim(F, p, g, raw, 777)
    with pytest.raises(F.FteError):
        same.load_state(blob[:-8])        # truncated
    bad = bytearray(blob)
    bad[0] ^= 0xFF
    with pytest.raises(F.FteError):
        same.load_state(bytes(bad))       # not a state blob
    same.load_state(blob)                 # the intact blob still loads
    same.step(10)
    same.close()
