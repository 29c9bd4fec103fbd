"""Launch graphs through the C ABI: the inject/step calls of a run recorded
with fte_capture_begin/fte_capture_end and replayed with fte_graph_launch
give the trajectories and sums of the same calls made directly, on every
replay; recording runs nothing and leaves the context where it began;
synchronising entry points are refused while recording; a graph only
launches from the state it was recorded at."""
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


def _case(n, precision):
    cfg = W.cir_time_dependent(n_particles=n, n_snap=8)
    # observers (ring bins in longitude) where the particles are within the
    # few hours the test steps: 0.15-0.35 au around the ecliptic
    obs = [(r * W.AU, 90 * W.DEG, 0.0, 0.05 * W.AU, 20 * W.DEG, 10 * W.DEG, 36) for r in (0.15, 0.25, 0.35)]
    p = dict(cfg["params"], precision=precision, observers=obs, n_t=12)
    inj = dict(cfg["injection"], n_total=n, pid0=0, k0=0, n_inj_steps=400)
    return cfg, p, cfg["grid"], inj


def _calls(sim, inj, n, chunks):
    """Continuous injection: every pid whose first step falls before the end
    of a chunk is injected before the chunk is stepped (as the benchmark
    does)."""
    done, injected = 0, 0
    for m in chunks:
        done += m
        j_max = min(n, int(math.ceil(done * n / inj["n_inj_steps"])) + 1)
        if j_max > injected:
            sim.inject(inj, j_max - injected, injected)
            injected = j_max
        sim.step(m)


def _state(sim, torch):
    torch.cuda.synchronize()
    out = sim.particles()
    m = out["status"] == 0
    o = np.argsort(out["pid"][m])
    sums, w = sim.read_hist()
    return {k: out[k][m][o] for k in ("pid", "x", "mu", "lnp", "w")}, sums, w, sim.stats()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_graph_replays_match_direct_calls(F, torch_cuda, precision):
    torch = torch_cuda
    n = 20000 if precision == "mixed" else 4000
    cfg, p, g, inj = _case(n, precision)
    vb = W.make_raw(g, cfg["wind"], xp=torch, device=torch.device("cuda:0"))
    per = int(g["dt_s"] / p["dt"])
    chunks = [150, per - 150, 2 * per + 37, 90]          # crosses compactions and snapshot intervals
    torch.cuda.synchronize()                            # the wind was made on the default stream
    side = torch.cuda.Stream()                          # capture needs a stream other than the default
    with torch.cuda.stream(side):
        sim = F.Simulation(p, g, n)
        sim.load_grid(vb)
        sim.set_launch(256, 64, 64, 1)
        _calls(sim, inj, n, chunks)
        ref, ref_sums, ref_w, ref_st = _state(sim, torch)
        assert (ref_sums > 0).sum() > 10

        sim.reset()
        sim.capture_begin()
        with pytest.raises(F.FteError):                 # a synchronising call is refused while recording
            sim.read_hist()
        _calls(sim, inj, n, chunks)
        graph = sim.capture_end()
        st = sim.stats()                                # nothing ran, the clock is back at the start
        assert st.global_step == 0 and st.particle_steps == 0
        for rep in range(3):
            sim.reset()
            sim.graph_launch(graph)
            with pytest.raises(F.FteError):             # launched again from the end state: refused
                sim.graph_launch(graph)
            got, sums, w, st = _state(sim, torch)
            print(f"replay {rep}: {len(got['pid'])} active particles, {st.particle_steps} particle-steps")
            assert st.global_step == sum(chunks)
            assert st.particle_steps == ref_st.particle_steps
            for key in ref:
                assert np.array_equal(ref[key], got[key]), (rep, key)
            assert w == pytest.approx(ref_w, rel=1e-14)     # atomic sums: order-dependent rounding
            sc = np.abs(ref_sums).max()
            assert np.allclose(sums, ref_sums, rtol=1e-12, atol=1e-14 * sc)
            sim.step(25)                                # direct work between the replays
            torch.cuda.synchronize()
        graph.close()
        sim.close()
