"""Batched ensembles through the C ABI: runs sharing one grid and one particle
population give, run by run, exactly the trajectories and observer sums of
separate single-run contexts (run id base + r, the run's lambda and kappa
ratio, its step count), one run also against the oracle directly; the
autotuner leaves the results unchanged."""
import numpy as np
import pytest

import fte_workloads as W
from cases import amr_cir_case

pytestmark = pytest.mark.gpu

AU = W.AU
DEG = W.DEG
RUNS = [dict(lambda_ref=0.05 * AU, kperp_ratio=0.05, n_steps=300),
        dict(lambda_ref=0.1 * AU, kperp_ratio=0.0, n_steps=150),
        dict(lambda_ref=0.3 * AU, kperp_ratio=0.02, n_steps=223)]
COUNTS = [(200, 1000), (131, 5000), (77, 9000)]


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
    p = dict(p, run_id=7)
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    return p, g, inj, raw


def _inj(inj, r):
    n, pid0 = COUNTS[r]
    return dict(inj, pid0=pid0, n_total=n, n_inj_steps=min(120, RUNS[r]["n_steps"]), run=r)


def _sorted(parts):
    o = np.argsort(parts["pid"])
    return {k: v[o] for k, v in parts.items()}


def _ensemble(F, p, g, raw, chunks, autotune_at=None, launch=(128, 25, 75, 2)):
    sim = F.Simulation(dict(p, runs=RUNS), g, sum(n for n, _ in COUNTS))
    sim.load_grid(raw)
    sim.set_launch(*launch)
    for r in range(len(RUNS)):
        i = _inj(p["_inj"], r)
        sim.inject(i, i["n_total"], i["pid0"])
    best = None
    for k, c in enumerate(chunks):
        if autotune_at is not None and k == autotune_at:
            best = sim.autotune(50)
        sim.step(c)
    out = dict(parts=_sorted(sim.particles()), hist=sim.read_hist(), j=sim.bin_observers()[0], st=sim.stats(),
               best=best)
    sim.close()
    return out


def test_ensemble_matches_single_runs(F, torch_cuda, orc):
    p, g, inj, raw = _case()
    p["_inj"] = inj
    # no compaction, so that finished runs stay held (status DONE) to the end
    E = _ensemble(F, p, g, raw, [100, 200], launch=(128, 25, 0, 0))
    sums, w = E["hist"]
    nb = len(p["observers"]) * p["n_e"] * p["n_t"] * p["n_batch"]
    assert E["j"].shape == (3, len(p["observers"]), p["n_e"], p["n_t"])
    done = 0
    for r, run in enumerate(RUNS):
        q = {k: v for k, v in p.items() if k != "_inj"}
        q.update(run_id=p["run_id"] + r, lambda_ref=run["lambda_ref"], kperp_ratio=run["kperp_ratio"])
        i = _inj(inj, r)
        i1 = dict(i, run=0)
        sim = F.Simulation(q, g, i["n_total"])
        sim.load_grid(raw)
        sim.set_launch(128, 25, 0, 0)
        sim.inject(i1, i["n_total"], i["pid0"])
        sim.step(run["n_steps"])
        S = _sorted(sim.particles())
        s_sums, s_w = sim.read_hist()
        sim.close()
        mine = (E["parts"]["pid"] >= i["pid0"]) & (E["parts"]["pid"] < i["pid0"] + i["n_total"])
        e = {k: v[mine] for k, v in E["parts"].items()}
        s = S
        assert np.array_equal(e["pid"], s["pid"]) and len(s["pid"]) == i["n_total"]
        # particles still active in the single run are DONE (or retired alike) in the ensemble
        act = s["status"] == 0
        assert np.all(e["status"][act] == 5)
        assert np.array_equal(e["status"][~act], s["status"][~act])
        done += int(act.sum())
        if run["kperp_ratio"] > 0:
            # same kernel instance as the single run: bit-identical
            for k in ("x", "mu", "lnp", "w", "kinj"):
                assert np.array_equal(e[k], s[k]), (r, k)
        else:
            # the single run uses the kernel without kappa_perp terms, the
            # ensemble the one with them at kappa_perp = 0: the same arithmetic
            # up to the compiler's rounding choices (the FP64 bar of the oracle
            # parity tests)
            assert np.array_equal(e["kinj"], s["kinj"]) and np.array_equal(e["w"], s["w"])
            assert np.abs(e["x"] - s["x"]).max() <= 1e-10 * AU
            assert np.abs(e["mu"] - s["mu"]).max() <= 1e-10
            assert np.abs(e["lnp"] - s["lnp"]).max() <= 1e-10 * np.abs(s["lnp"]).max()
        assert w[r] == pytest.approx(s_w, rel=1e-14)
        blk = sums[r * nb:(r + 1) * nb]
        sc = max(np.abs(s_sums).max(), 1e-300)
        assert np.allclose(blk, s_sums, rtol=1e-12, atol=1e-14 * sc), r
        if r == 1:
            # and this run against the oracle directly
            G = orc.Grid(g, raw)
            P = orc.inject(q, i1, i["n_total"], i["pid0"])
            orc.run(q, G, P, 0, run["n_steps"], None)
            o = np.argsort(P.pid)
            live = P.status[o] == 0
            sel = np.isin(e["pid"], P.pid[o][live])
            assert np.allclose(e["x"][sel], P.x[o][live], rtol=0, atol=1e-10 * AU)
    assert E["st"].n_retired[5] == done > 0


def test_autotune_leaves_results_unchanged(F, torch_cuda):
    p, g, inj, raw = _case()
    p["_inj"] = inj
    A = _ensemble(F, p, g, raw, [100, 200])
    B = _ensemble(F, p, g, raw, [100, 200], autotune_at=1)
    block, spl, compact = B["best"]
    assert block in (64, 128, 256) and spl == 25 and compact % spl == 0
    assert np.array_equal(A["parts"]["pid"], B["parts"]["pid"])
    for k in ("x", "mu", "lnp", "status"):
        assert np.array_equal(A["parts"][k], B["parts"][k]), k
    sa, sb = A["hist"][0], B["hist"][0]
    assert np.allclose(sa, sb, rtol=1e-12, atol=1e-14 * max(np.abs(sa).max(), 1e-300))
    assert A["st"].particle_steps == B["st"].particle_steps
