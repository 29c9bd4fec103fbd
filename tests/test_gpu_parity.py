"""Parity of the HIP path (through the C ABI) with the FP64 CPU oracle.

FP64 path: every trajectory within 1e-10 relative of the oracle's (positions
scaled by 1 au, ln p by max(|ln p|, 1)), identical statuses, observer batch sums
within 1e-9 relative.  Mixed path: statistical agreement.  Sizes span several
blocks and leaves, ragged particle counts and launch shapes."""
import math

import numpy as np
import pytest

import fte_workloads as W
from cases import amr_cir_case, near_observers

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


def gpu_run(F, torch, p, g, raw, injs, n_steps, launch=(256, 64, 512), step_chunks=None):
    n_tot = sum(n for _, n, _ in injs)
    sim = F.Simulation(p, g, max(n_tot, 1))
    sim.load_grid(raw)
    sim.set_launch(*launch)
    for inj, n, first in injs:
        sim.inject(inj, n, first)
    chunks = step_chunks or [n_steps]
    for c in chunks:
        sim.step(c)
    torch.cuda.synchronize()
    out = sim.particles()
    sums, w = sim.read_hist()
    st = sim.stats()
    sim.close()
    return out, sums, w, st


def oracle_run(orc, p, g, raw, injs, n_steps):
    G = orc.Grid(g, raw)
    parts = []
    for inj, n, first in injs:
        parts.append(orc.inject(p, inj, n, first))
    P = parts[0]
    for q in parts[1:]:
        for k in ("x", "mu", "lnp", "w", "pid", "kinj", "status"):
            setattr(P, k, np.concatenate([getattr(P, k), getattr(q, k)]))
    h = np.zeros(orc.hist_size(p))
    orc.run(p, G, P, 0, n_steps, h)
    return P, h


def compare(got, ref, sums, h, tol=1e-10, hist_tol=1e-9):
    """Held GPU particles (live, or retired since the last compaction) against
    the oracle's particles of the same pid; every particle the oracle still has
    active must be held by the GPU."""
    rpos = {int(k): i for i, k in enumerate(ref.pid)}
    idx = np.array([rpos[int(k)] for k in got["pid"]], dtype=np.int64)
    assert len(np.unique(got["pid"])) == len(got["pid"]), "duplicate pids"
    live = set(int(k) for k in ref.pid[ref.status == 0])
    assert live <= set(int(k) for k in got["pid"]), "an active particle is missing"
    dx = np.abs(got["x"] - ref.x[idx]) / np.maximum(np.abs(ref.x[idx]), AU)
    dmu = np.abs(got["mu"] - ref.mu[idx])
    rl = ref.lnp[idx]
    dl = np.abs(got["lnp"] - rl) / np.maximum(np.abs(rl), 1.0)
    assert np.array_equal(got["status"], ref.status[idx])
    assert np.array_equal(got["kinj"], ref.kinj[idx])
    assert np.allclose(got["w"], ref.w[idx], rtol=1e-12, atol=0)
    worst = max(dx.max(initial=0), dmu.max(initial=0), dl.max(initial=0))
    assert worst <= tol, (dx.max(initial=0), dmu.max(initial=0), dl.max(initial=0))
    scale = max(np.abs(h).max(), 1e-300)
    bad = np.abs(sums - h) > hist_tol * np.maximum(np.abs(h), scale * 1e-6)
    assert bad.sum() == 0, (bad.sum(), np.abs(sums - h).max() / scale)
    return worst


def test_tiny_parker_fp64_parity(F, torch_cuda, orc):
    """The tiny Parker workload (uniform 64x32x64 grid, 2,000 protons,
    100 keV, power-law D_mumu) over its full 5,000 steps (13.9 h)."""
    cfg = W.tiny_parker()
    p = near_observers(dict(cfg["params"], precision="fp64"))
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"])
    injs = [(cfg["injection"], 2000, 0)]
    got, sums, w, st = gpu_run(F, torch_cuda, p, g, raw, injs, 5000)
    ref, h = oracle_run(orc, p, g, raw, injs, 5000)
    worst = compare(got, ref, sums, h)
    print("tiny parker worst relative deviation", worst)
    assert w == pytest.approx(ref.w.sum(), rel=1e-14)
    assert st.n_live >= (ref.status == 0).sum()
    for k in range(1, 5):
        assert st.n_retired[k] == (ref.status == k).sum()
    assert (h > 0).sum() > 50, "observers saw too little: the test would be vacuous"
    # finalize kernel against the oracle's finalisation of the same sums
    sim = F.Simulation(p, g, 2000)
    sim.load_grid(raw)
    sim.inject(cfg["injection"], 2000, 0)
    sim.step(5000)
    jg, sg = sim.bin_observers()
    sums2, w2 = sim.read_hist()
    sim.close()
    jo, so = orc.finalize(p, sums2, w2)
    assert np.allclose(jg, jo, rtol=1e-12, atol=0) and np.allclose(sg, so, rtol=1e-10, atol=1e-300)


def test_amr_cir_kperp_fp64_parity(F, torch_cuda, orc):
    """3-level AMR, stretched radius, 3 snapshots of a CIR wind, Eq. 5
    D_mumu, kappa_perp, continuous injection split over two calls (ragged
    count 777), compaction between launches."""
    p, g, inj = amr_cir_case()
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    injs = [(inj, 400, 1000), (inj, 377, 1400)]
    got, sums, w, st = gpu_run(F, torch_cuda, p, g, raw, injs, 300, launch=(128, 25, 75))
    ref, h = oracle_run(orc, p, g, raw, injs, 300)
    worst = compare(got, ref, sums, h)
    print("amr cir worst relative deviation", worst)
    assert (ref.status != 0).sum() > 0 and (ref.status == 0).sum() > 100


def test_records_match_oracle(F, torch_cuda, orc):
    """Every record of the ghost-padded blocks (interior: derived fields;
    ghost layer: the block-boundary rule) equals the oracle's value of the
    same level-L cell centre."""
    p, g, _ = amr_cir_case()
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    sim = F.Simulation(p, g, 16)
    sim.load_grid(raw)
    rec = sim.records().cpu().numpy()
    sim.close()
    G = orc.Grid(g, raw)
    rng = np.random.default_rng(0)
    bx = g["bx"]
    px = [b + 2 for b in bx]
    nf = 13 if rec.shape[-1] == 13 else 10
    scale = np.abs(rec[..., :nf]).reshape(-1, nf).max(axis=0)
    n = 0
    for leaf in rng.choice(len(g["leaves"]), size=40, replace=False):
        L, I, J, K = g["leaves"][leaf]
        for _ in range(40):
            loc = [rng.integers(-1, bx[a] + 1) for a in range(3)]
            pc = (loc[0] + 1) + px[0] * ((loc[1] + 1) + px[1] * (loc[2] + 1))
            c = np.array([I * bx[0] + loc[0], J * bx[1] + loc[1], K * bx[2] + loc[2]])
            snap = int(rng.integers(0, g["n_snap"]))
            want = G.derived_virtual(snap, int(L), c)[:nf]
            gotv = rec[snap, leaf, pc, :nf]
            assert np.all(np.abs(gotv - want) <= 1e-11 * scale + 1e-12 * np.abs(want)), (leaf, loc, snap)
            n += 1
    assert n == 1600


def test_launch_shape_invariance(F, torch_cuda):
    """Trajectories depend only on (pid, step): block size, steps per launch,
    compaction and how the steps are split across calls change nothing."""
    cfg = W.tiny_parker(n_particles=3001)
    p = dict(cfg["params"], precision="fp64", r_in=0.098 * AU)
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"])
    injs = [(dict(cfg["injection"], n_total=3001), 3001, 0)]
    a, sa, _, _ = gpu_run(F, torch_cuda, p, g, raw, injs, 240, launch=(256, 64, 0))
    ma = a["status"] == 0
    oa = np.argsort(a["pid"][ma])
    for launch, chunks in (((64, 1, 7, 1), [13, 100, 127]), ((128, 8, 16, 0), [240]), ((192, 5, 15, 1), [1, 239])):
        b, sb, _, _ = gpu_run(F, torch_cuda, p, g, raw, injs, 240, launch=launch, step_chunks=chunks)
        mb = b["status"] == 0
        ob = np.argsort(b["pid"][mb])
        for k in ("x", "mu", "lnp", "pid"):
            assert np.array_equal(a[k][ma][oa], b[k][mb][ob]), (launch, k)
        assert np.allclose(sa, sb, rtol=1e-12, atol=0)


@pytest.mark.parametrize("kperp", [0.0, 0.05])
def test_mixed_time_dependent_launch_shape_invariance(F, torch_cuda, kperp):
    """The float kernel's unrolled two-snapshot gather (plain and cross-field
    records) on a 3-level time-dependent grid: trajectories depend only on
    (pid, step), bit for bit, whatever the block size, steps per launch,
    compaction, spatial sort and call splitting."""
    p, g, inj = amr_cir_case(kperp=kperp)
    p = dict(p, precision="mixed")
    r, th, ph = W.cell_centres(g)
    raw = np.stack([W.cir_wind(r, th, ph, k * g["dt_s"], width=25 * DEG) for k in range(g["n_snap"])])
    injs = [(inj, 400, 1000), (inj, 377, 1400)]
    runs = []
    for launch, chunks in (((256, 64, 64, 1), [300]), ((64, 16, 32, 1), [100, 200]), ((128, 25, 75, 0), [300]),
                           ((192, 5, 15, 1), [1, 299])):
        got, sums, w, st = gpu_run(F, torch_cuda, p, g, raw, injs, 300, launch=launch, step_chunks=chunks)
        m = got["status"] == 0
        o = np.argsort(got["pid"][m])
        runs.append(({k: got[k][m][o] for k in ("x", "mu", "lnp", "pid", "w")}, sums, launch))
    a, sa, _ = runs[0]
    assert len(a["pid"]) > 300
    for b, sb, launch in runs[1:]:
        for k in ("pid", "x", "mu", "lnp", "w"):
            assert np.array_equal(a[k], b[k]), (launch, k)
        assert np.allclose(sa, sb, rtol=1e-12, atol=1e-12 * np.abs(sa).max())


def test_cir_grid_launch_shape_invariance(F, torch_cuda):
    """The mixed path on the CIR grid (16x12x16 blocks, so a workgroup's LDS
    record tile holds 3 of a leaf's 18 padded k-layers and many corners come
    from L1 instead): trajectories bit-identical across block sizes, steps per
    launch and compaction intervals, which change every workgroup's
    composition, tile anchor and so which gathers read LDS."""
    torch = torch_cuda
    cfg = W.cir_time_dependent(n_particles=3_000_000, n_snap=5)
    g = cfg["grid"]
    dev = torch.device("cuda:0")
    raw = W.make_raw(g, cfg["wind"], xp=torch, device=dev)
    N, S = cfg["n_particles"], cfg["injection"]["n_inj_steps"]
    inj = cfg["injection"]
    p = dict(cfg["params"], precision="mixed")
    runs = []
    for launch in ((256, 64, 64, 1), (128, 32, 64, 1), (192, 16, 48, 1)):
        sim = F.Simulation(p, g, 250_000)
        sim.load_grid(raw)
        sim.set_launch(*launch)
        injected, n0 = 0, 0
        for chunk in (564, 564):
            n1 = n0 + chunk
            j_max = min(N, int(math.ceil(n1 * N / S)) + 1)
            sim.inject(inj, j_max - injected, injected)
            injected = j_max
            sim.step(chunk)
            n0 = n1
        torch.cuda.synchronize()
        got = sim.particles()
        assert sim.stats().device_flags == 0
        sim.close()
        m = got["status"] == 0
        o = np.argsort(got["pid"][m])
        runs.append(({k: got[k][m][o] for k in ("pid", "x", "mu", "lnp")}, launch))
    a, _ = runs[0]
    assert len(a["pid"]) > 100_000
    for b, launch in runs[1:]:
        for k in ("pid", "x", "mu", "lnp"):
            assert np.array_equal(a[k], b[k]), (launch, k)


def test_edge_cases(F, torch_cuda):
    torch = torch_cuda
    cfg = W.tiny_parker(n_particles=100)
    p = dict(cfg["params"], precision="fp64")
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"])
    sim = F.Simulation(p, g, 100)
    with pytest.raises(F.FteError):          # step before load
        sim.step(1)
    sim.load_grid(raw)
    sim.step(10)                             # no particles: fine
    sim.inject(cfg["injection"], 0, 0)       # empty injection: fine
    sim.step(0)
    with pytest.raises(F.FteError) as e:     # over capacity
        sim.inject(cfg["injection"], 101, 0)
    assert e.value.status == F.FTE_ENOMEM
    sim.inject(cfg["injection"], 100, 0)
    sim.step(5)
    torch.cuda.synchronize()
    st = sim.stats()
    assert st.n_live == 100 and st.particle_steps == 500 and st.global_step == 15
    bad = raw.copy()
    bad[0, 3, 7, 2] = np.nan
    with pytest.raises(F.FteError):
        sim.load_grid(bad)
    sim.close()
    # steps past the last snapshot of a time-dependent grid
    p2, g2, _ = amr_cir_case(n_levels=1, kperp=0.0, n_snap=2)
    r, th, ph = W.cell_centres(g2)
    raw2 = np.stack([W.cir_wind(r, th, ph, k * g2["dt_s"]) for k in range(2)])
    sim2 = F.Simulation(p2, g2, 10)
    sim2.load_grid(raw2)
    sim2.step(int(g2["dt_s"] / p2["dt"]) + 1)
    with pytest.raises(F.FteError) as e:
        sim2.step(1)
    assert e.value.status == F.FTE_ERANGE
    sim2.close()


def test_all_absorbed_then_continue(F, torch_cuda, orc):
    """Every particle leaves through the inner sphere; compaction empties
    the store; stepping and injecting go on."""
    cfg = W.tiny_parker(n_particles=500)
    p = dict(cfg["params"], precision="fp64", r_in=0.1 * AU * (1 - 1e-9), dmm_model="iso", lambda_ref=1e6)
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"])
    inj = dict(cfg["injection"], n_total=500)
    sim = F.Simulation(p, g, 500)
    sim.load_grid(raw)
    sim.set_launch(256, 16, 32)
    sim.inject(inj, 250, 0)
    sim.step(2000)
    sim.inject(inj, 250, 250)
    sim.step(100)
    torch_cuda.cuda.synchronize()
    st = sim.stats()
    got = sim.particles()
    sim.close()
    G = orc.Grid(g, raw)
    a = orc.inject(p, inj, 250, 0)
    orc.run(p, G, a, 0, 2000)
    b = orc.inject(p, inj, 250, 250)
    orc.run(p, G, b, 2000, 100)
    assert st.n_retired[1] == (a.status == 1).sum() + (b.status == 1).sum()
    assert st.n_live == len(got["pid"])
    assert (got["status"] == 0).sum() == (a.status == 0).sum() + (b.status == 0).sum()


def test_mixed_path_statistics(F, torch_cuda, orc):
    """Mixed precision (float records and step arithmetic, double position,
    time and radial tests) against the FP64 oracle on the tiny Parker
    workload: trajectories driven by the same noise stay close and every
    observer bin agrees within 3 standard errors."""
    cfg = W.tiny_parker()
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"])
    injs = [(cfg["injection"], 2000, 0)]
    pm = near_observers(dict(cfg["params"], precision="mixed"))
    got, sums, w, _ = gpu_run(F, torch_cuda, pm, g, raw, injs, 5000)
    p64 = near_observers(dict(cfg["params"], precision="fp64"))
    ref, h = oracle_run(orc, p64, g, raw, injs, 5000)
    both = np.intersect1d(got["pid"], ref.pid[ref.status == 0])
    assert len(both) > 0.8 * (ref.status == 0).sum()
    gi = np.searchsorted(np.sort(got["pid"]), both)
    og = np.argsort(got["pid"])
    ri = np.argsort(ref.pid)
    rsel = ri[np.searchsorted(ref.pid[ri], both)]
    dx = np.linalg.norm(got["x"][og][gi] - ref.x[rsel], axis=1) / AU
    print("mixed: median |dx| au", np.median(dx), "p99", np.quantile(dx, 0.99))
    assert np.median(dx) < 1e-3
    jg, sg = orc.finalize(p64, sums, w)
    jo, so = orc.finalize(p64, h, ref.w.sum())
    sig = np.sqrt(sg ** 2 + so ** 2)
    m = (jo > 0) | (jg > 0)
    z = np.abs(jg - jo)[m] / np.maximum(sig[m], 1e-300)
    assert np.all(z < 3.0), z.max()
    assert abs(jg.sum() / jo.sum() - 1) < 0.01


def test_full_size_cir_sampled(F, torch_cuda, orc):
    """The CIR workload at full size (2,346 leaves, 48 snapshots, 10^7
    particle store, the benchmark's launch shape and lazy continuous
    injection) for 1,200 steps: 48 sampled particles re-run one by one in the
    oracle agree to 1e-10 on the FP64 path; the mixed path on the same sample
    stays within a small drift."""
    torch = torch_cuda
    n_steps = 1200
    cfg = W.cir_time_dependent()
    g = cfg["grid"]
    dev = torch.device("cuda:0")
    raw = W.make_raw(g, cfg["wind"], xp=torch, device=dev)
    N, S = cfg["n_particles"], cfg["injection"]["n_inj_steps"]
    inj = cfg["injection"]
    held = {}
    for prec in ("fp64", "mixed"):
        p = dict(cfg["params"], precision=prec)
        sim = F.Simulation(p, g, N)
        sim.load_grid(raw)
        sim.set_launch(256, 64, 64, 1)
        injected, n0 = 0, 0
        for chunk in (564, 564, n_steps - 1128):
            n1 = n0 + chunk
            j_max = min(N, int(math.ceil(n1 * N / S)) + 1)
            sim.inject(inj, j_max - injected, injected)
            injected = j_max
            sim.step(chunk)
            n0 = n1
        torch.cuda.synchronize()
        held[prec] = sim.particles()
        st = sim.stats()
        assert st.device_flags == 0
        sim.close()
    # sample among particles that started before step 1,100
    rng = np.random.default_rng(5)
    j_hi = int(1100 * N / S)
    sample = np.sort(rng.choice(j_hi, size=48, replace=False))
    k_hi = int(math.floor(n_steps * cfg["params"]["dt"] / g["dt_s"])) + 2
    G = orc.Grid(g, raw[: k_hi + 1].cpu().numpy())
    p64 = dict(cfg["params"], precision="fp64")
    ref = [orc.inject(p64, inj, 1, int(j)) for j in sample]
    for q in ref:
        orc.run(p64, G, q, 0, n_steps, None, 1)
    for prec, tol in (("fp64", 1e-10), ("mixed", None)):
        got = held[prec]
        pos = {int(k): i for i, k in enumerate(got["pid"])}
        drift = []
        for j, q in zip(sample, ref):
            if int(j) not in pos:
                assert q.status[0] != 0, (prec, j)       # retired and compacted away
                continue
            i = pos[int(j)]
            if tol is not None:
                assert got["status"][i] == q.status[0], (j, got["status"][i], q.status[0])
                dx = np.abs(got["x"][i] - q.x[0]).max() / max(np.abs(q.x[0]).max(), AU)
                assert dx < tol and abs(got["mu"][i] - q.mu[0]) < tol, (j, dx)
                assert abs(got["lnp"][i] - q.lnp[0]) < tol * max(1.0, abs(q.lnp[0]))
            elif got["status"][i] == 0 and q.status[0] == 0:
                drift.append(np.linalg.norm(got["x"][i] - q.x[0]) / AU)
        if tol is None:
            assert len(drift) > 20 and np.median(drift) < 1e-3, drift
