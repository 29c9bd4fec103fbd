"""Snapshot streaming through the C ABI: a grid held as a ring of three
snapshot slots, filled with fte_load_snapshot as the clock advances, gives
the records, trajectories and observer sums of the fully loaded grid; steps
that reach a snapshot not yet loaded are refused."""
import numpy as np
import pytest

import fte_workloads as W
from cases import amr_cir_case

pytestmark = pytest.mark.gpu

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


def test_ring_of_slots_matches_full_grid(F, torch_cuda):
    torch = torch_cuda
    p, g, inj = amr_cir_case(n_snap=6)
    p = dict(p, t0=0.0, n_t=14, dT=1300.0)
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    per = int(g["dt_s"] / p["dt"])                   # steps per snapshot interval
    n_steps = 5 * per - 7

    a = F.Simulation(p, g, 777)
    a.load_grid(raw)
    a.set_launch(128, 25, 75, 2)
    a.inject(inj, 777, 1000)
    rec_full = a.records().cpu().numpy()
    a.step(n_steps)
    A = a.particles()
    sa, wa = a.read_hist()
    a.close()

    vb = torch.from_numpy(raw).to("cuda:0").contiguous()
    gs = dict(g, n_slots=3)
    b = F.Simulation(p, gs, 777)
    b.set_launch(128, 25, 75, 2)
    b.load_snapshot(0, vb)
    b.load_snapshot(1, vb)
    b.inject(inj, 777, 1000)
    done = 0
    for k in range(5):
        if k > 0:
            with pytest.raises(F.FteError):          # snapshot k+1 is not resident yet
                b.step(1)
            b.load_snapshot(k + 1, vb)
            rec = b.records().cpu().numpy()
            assert np.array_equal(rec[(k + 1) % 3], rec_full[k + 1])
        m = min((k + 1) * per, n_steps) - done
        b.step(m)
        done += m
    assert done == n_steps
    B = b.particles()
    sb, wb = b.read_hist()
    b.close()
    # compaction runs at other global steps when the steps come in other
    # chunks, so compare the particles still active (retired ones may be held
    # or already dropped)
    ma, mb = A["status"] == 0, B["status"] == 0
    oa, ob = np.argsort(A["pid"][ma]), np.argsort(B["pid"][mb])
    for key in ("pid", "x", "mu", "lnp"):
        assert np.array_equal(A[key][ma][oa], B[key][mb][ob]), key
    assert wa == pytest.approx(wb, rel=1e-14)      # atomic sums: order-dependent rounding
    sc = max(np.abs(sa).max(), 1e-300)
    assert (sa > 0).sum() > 20
    assert np.allclose(sa, sb, rtol=1e-12, atol=1e-14 * sc)
