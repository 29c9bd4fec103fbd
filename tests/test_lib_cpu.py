"""Host-side checks of the C-ABI library that need no GPU: it loads, exports
every symbol include/fte.h declares, and its grid validation and buffer sizing
(pure host logic) accept valid descriptions and reject broken ones."""
import os
import re

import numpy as np
import pytest

import fte_workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def F():
    from paper_2404_12164_amd import fte
    if not os.path.exists(fte.LIB_PATH):
        from paper_2404_12164_amd import build
        build.build()
    fte.lib()
    return fte


def test_exports_every_declared_symbol(F):
    hdr = open(os.path.join(ROOT, "include", "fte.h")).read()
    declared = set(re.findall(r"\b(fte_[a-z_]+)\s*\(", hdr))
    assert declared == set(F.SYMBOLS)
    L = F.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_struct_sizes_match_header_layout(F):
    import ctypes as C
    # the binding's structures are laid out like the C ones (natural alignment)
    assert C.sizeof(F.fte_observer) == 64
    assert C.sizeof(F.fte_sizes) == 48
    assert C.sizeof(F.fte_buffers) == 64
    assert C.sizeof(F.fte_injection) == 8 * 9 + 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8 + 8 + 8
    assert C.sizeof(F.fte_run) == 24


def test_query_sizes_valid(F):
    cfg = W.tiny_parker()
    s = F.fte_query_sizes(cfg["params"], cfg["grid"], 2000)
    pc = 18 ** 3
    assert s.grid_bytes == 1 * 32 * pc * 10 * 8          # stride 10 without kappa_perp
    mixed = dict(cfg["params"], precision="mixed")
    assert F.fte_query_sizes(mixed, cfg["grid"], 2000).grid_bytes == s.grid_bytes // 2
    assert s.hist_bytes == 1 * 10 * 60 * 32 * 8
    assert s.state_bytes >= 2000 * 64


def test_query_sizes_amr_cir(F):
    cfg = W.cir_time_dependent(n_particles=1000, n_snap=3)
    s = F.fte_query_sizes(cfg["params"], cfg["grid"], 1000)
    nl = len(cfg["grid"]["leaves"])
    assert s.grid_bytes == 3 * nl * 18 * 14 * 18 * 10 * 4
    kp = dict(cfg["params"], kperp_ratio=0.01)
    assert F.fte_query_sizes(kp, cfg["grid"], 1000).grid_bytes == 3 * nl * 18 * 14 * 18 * 13 * 4


def _tiny_grid(**over):
    n1, bx = (16, 8, 16), (4, 4, 4)
    g = W.grid_desc(0, 0.1 * W.AU, 0.1 * W.AU, 30 * W.DEG, 15 * W.DEG, 0.0, 2 * np.pi / 16, n1, bx,
                    W.uniform_leaves(n1, bx), 1)
    g.update(over)
    return g


def test_rejects_broken_grids(F):
    p = W.tiny_parker()["params"]
    ok = _tiny_grid()
    F.fte_query_sizes(p, ok, 10)
    bad = []
    bad.append(_tiny_grid(leaves=ok["leaves"][:-1]))                       # hole
    dup = np.concatenate([ok["leaves"], ok["leaves"][:1]])
    bad.append(_tiny_grid(leaves=dup))                                      # overlap
    bad.append(_tiny_grid(bx=[3, 4, 4], n1=[15, 8, 16]))                   # odd block
    bad.append(_tiny_grid(dph=0.1))                                         # periodic span wrong
    bad.append(_tiny_grid(dxi=-1.0))
    bad.append(_tiny_grid(n_snap=0))
    lv = ok["leaves"].copy()
    lv[0, 0] = 2
    bad.append(_tiny_grid(leaves=lv))                                       # level out of range
    for g in bad:
        with pytest.raises(F.FteError):
            F.fte_query_sizes(p, g, 10)


def test_rejects_unbalanced_amr(F):
    p = W.tiny_parker()["params"]
    n1, bx = (16, 8, 16), (4, 4, 4)
    # refine one level-1 block twice without refining its neighbours
    leaves = []
    nb = [n1[a] // bx[a] for a in range(3)]
    for K in range(nb[2]):
        for J in range(nb[1]):
            for I in range(nb[0]):
                if (I, J, K) != (1, 0, 1):
                    leaves.append((1, I, J, K))
    for d in range(8):
        a, b, c = 2 + (d & 1), 0 + ((d >> 1) & 1), 2 + ((d >> 2) & 1)
        if d != 7:
            leaves.append((2, a, b, c))
        else:
            for e in range(8):
                leaves.append((3, 2 * a + (e & 1), 2 * b + ((e >> 1) & 1), 2 * c + ((e >> 2) & 1)))
    g = W.grid_desc(0, 0.1 * W.AU, 0.1 * W.AU, 30 * W.DEG, 15 * W.DEG, 0.0, 2 * np.pi / 16, n1, bx,
                    np.array(leaves, np.int32), 3)
    with pytest.raises(F.FteError):
        F.fte_query_sizes(p, g, 10)
    # the balanced version of the same refinement is accepted
    marks = {(1, 1, 0, 1), (2, 3, 1, 3)}
    g2 = W.grid_desc(0, 0.1 * W.AU, 0.1 * W.AU, 30 * W.DEG, 15 * W.DEG, 0.0, 2 * np.pi / 16, n1, bx,
                     W.amr_leaves(n1, bx, 3, lambda L, I, J, K: (L, I, J, K) in marks), 3)
    F.fte_query_sizes(p, g2, 10)


def test_rejects_bad_params(F):
    cfg = W.tiny_parker()
    for over in (dict(dt=0.0), dict(mass=-1.0), dict(n_batch=0), dict(n_batch=65), dict(dmm_model=7),
                 dict(q=2.5), dict(r_out=0.0), dict(run_id=70000), dict(precision=3),
                 dict(kink_sigma=float("nan")), dict(kink_sigma=float("-inf"))):
        with pytest.raises(F.FteError):
            F.fte_query_sizes(dict(cfg["params"], **over), cfg["grid"], 10)


def test_ensemble_sizes_and_rejections(F):
    cfg = W.tiny_parker()
    p = cfg["params"]
    runs = [dict(lambda_ref=0.1 * W.AU, kperp_ratio=0.01, n_steps=100), dict(lambda_ref=0.2 * W.AU, n_steps=50)]
    one = F.fte_query_sizes(p, cfg["grid"], 100)
    two = F.fte_query_sizes(dict(p, runs=runs), cfg["grid"], 100)
    assert two.hist_bytes == 2 * one.hist_bytes              # sums per run
    assert two.grid_bytes == one.grid_bytes // 10 * 13       # a run with kappa_perp: 13-field records
    bad = [[dict(lambda_ref=-1.0, n_steps=5)], [dict(lambda_ref=1e10, n_steps=0)],
           [dict(lambda_ref=1e10, kperp_ratio=-0.1, n_steps=5)], [dict(lambda_ref=1e10, n_steps=5)] * 65]
    for r in bad:
        with pytest.raises(F.FteError):
            F.fte_query_sizes(dict(p, runs=r), cfg["grid"], 100)
    with pytest.raises(F.FteError):        # ensembles do not combine with smoothing
        F.fte_query_sizes(dict(p, runs=runs, smoothing=dict(sigma_x=1e9, sigma_lne=0.1, sigma_t=60.0)),
                          cfg["grid"], 100)
    with pytest.raises(F.FteError):        # run ids must fit 16 bits
        F.fte_query_sizes(dict(p, runs=runs, run_id=65535), cfg["grid"], 100)


def test_streaming_grid_sizes(F):
    cfg = W.cir_time_dependent(n_particles=1000, n_snap=12)
    g = cfg["grid"]
    full = F.fte_query_sizes(cfg["params"], g, 1000)
    ring = F.fte_query_sizes(cfg["params"], dict(g, n_slots=3), 1000)
    assert ring.grid_bytes * 12 == full.grid_bytes * 3          # three snapshot slots
    assert F.fte_query_sizes(cfg["params"], dict(g, n_slots=40), 1000).grid_bytes == full.grid_bytes
    for bad in (1, -2):
        with pytest.raises(F.FteError):
            F.fte_query_sizes(cfg["params"], dict(g, n_slots=bad), 1000)


def test_largest_workload_sizes(F):
    """The largest workload (shocked CIR, 3 levels, 96 snapshots, kappa_perp,
    10^8 particles) validates, and its buffers fit one GPU's 288 GB: records
    of 13 floats per padded cell for every snapshot, the particle state twice
    (compaction ping-pong), the 5 x 20 x 288 x 32 observer sums."""
    cfg = W.cir_largest()
    g, p = cfg["grid"], cfg["params"]
    s = F.fte_query_sizes(p, g, cfg["n_particles"])
    nl = len(g["leaves"])
    assert s.grid_bytes == 96 * nl * 18 * 10 * 18 * 13 * 4
    assert s.hist_bytes >= 5 * 20 * 288 * 32 * 8
    total = s.grid_bytes + s.index_bytes + 2 * s.state_bytes + s.hist_bytes + s.work_bytes
    print("largest workload: grid", s.grid_bytes / 1e9, "GB, state", s.state_bytes / 1e9, "GB, total",
          total / 1e9, "GB")
    assert total < 120e9


def test_shocked_cir_jump_conditions():
    """The shocked CIR wind: across each shock the speed normal to the
    corotating pattern (V_r - U along the spiral's normal) drops by the
    compression ratio 3, upstream is the slow (forward shock) or fast
    (reverse shock) wind, and the stream interface between them is
    compressive too."""
    U, Vs, Vf = 500e3, 330e3, 650e3
    deg = W.DEG
    r = np.full(7, 1.0 * W.AU)
    th = np.full(7, 90 * deg)
    # psi = phi at t = 0 and r = r_B; move phi at r = r_B = 0.1 au instead
    rb = np.full(7, 0.1 * W.AU)
    ph = np.array([55, 59, 61, 67.5, 74, 76, 80]) * deg
    # a narrow interface keeps its tanh tails off the shocks' sides
    V = W.cir_shocked_wind(rb, th, ph, 0.0, width_if=0.1 * deg)[:, 0]
    assert V[0] == pytest.approx(Vf, rel=5e-4) and V[-1] == pytest.approx(Vs, rel=5e-4)   # rarefaction tails
    assert (V[1] - U) / (V[2] - U) == pytest.approx(3.0, rel=2e-3)         # reverse shock at 60 deg
    assert (V[5] - U) / (V[4] - U) == pytest.approx(3.0, rel=2e-3)         # forward shock at 75 deg
    assert V[2] > V[3] > V[4]                                              # interface, compressive
    # the pattern is a spiral of speed U: at 1 au the same jumps sit at
    # longitudes shifted by omega (r - r_B) / U
    shift = W.OMEGA_CIR * (0.9 * W.AU) / U
    V1 = W.cir_shocked_wind(r, th, ph - shift, 0.0, width_if=0.1 * deg)[:, 0]
    assert (V1[1] - U) / (V1[2] - U) == pytest.approx(3.0, rel=2e-3)
    assert (V1[5] - U) / (V1[4] - U) == pytest.approx(3.0, rel=2e-3)


def test_sort_workspace_bounded_by_particles(F):
    """The spatial sort's key space is bounded by the particle capacity, not
    by the grid: on the paper's 4-level grid (76,509 leaves, 2.35 x 10^8 leaf
    cells) the work buffer grows with capacity by O(bytes per particle) and
    holds no per-cell counter array beyond the load-time workspace."""
    cfg = W.paper_cir(n_levels=4, n_particles=1000)
    g = cfg["grid"]
    nl = len(g["leaves"])
    cells = nl * int(np.prod(g["bx"]))
    pc = int(np.prod(np.asarray(g["bx"]) + 2))
    cart = nl * pc * 6 * 8                       # load-time Cartesian (V, b) of one snapshot
    small = F.fte_query_sizes(cfg["params"], g, 10_000).work_bytes
    big = F.fte_query_sizes(cfg["params"], g, 1_000_000).work_bytes
    assert cells * 4 > 9e8                      # a per-cell count array would be ~1 GB
    assert small < cart + 4e6                   # keys + counts of at most 2^16 keys + the rest
    assert big - small < 1_000_000 * 4 * 5      # keys (4 B) + counts (4 per particle x 4 B) per particle
