"""Throughput benchmark of the focused-transport pseudo-particle path on one MI355X.

Workload (default): the time-dependent CIR wind - 48 hourly snapshots on a
stretched 256 x 60 x 192 grid with one extra AMR level in the compression band,
10^7 protons of 5-50 keV (E^-4) injected continuously at 0.1 au over 47 h,
16,920 steps of 10 s, three observers at 1 au, mixed precision (float records
and step arithmetic, double position/time/radial tests).  A bench "step" is one
fte_step_n call of `chunk` global steps (including the injection of the
particles that start in it, observer accumulation and compaction); the default
30 steps cover the whole 16,920-step run.  Prints one JSON line.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("fte_kernels.hip", "fte_device.hpp", "fte_internal.hpp"):
        h.update(open(os.path.join(ROOT, "paper_2404_12164_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def read_counters(name, kernel):
    """Per-particle-step figures of a step-kernel instance from a committed
    counter summary (profiles/), if they were taken on the current kernel
    source; None otherwise."""
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256_16") != kernel_source_hash() or kv.get("kernel") != kernel:
        return None
    out = {}
    for k, v in kv.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def advance(sim, injections, injected, n0, n1, every):
    """Steps n0 .. n1 of continuous injections (one per run) on `sim`.
    Before each stretch of steps up to the next multiple of `every`, every
    pid of every injection whose first step can fall before the stretch's end
    is injected (injected[r] counts run r's pids so far).  A pid injected
    ahead of its first step holds a lane of the waves that step the others
    until then, so the injection keeps pace with the launches rather than
    with the caller's chunks."""
    while n0 < n1:
        n2 = min(n1, (n0 // every + 1) * every)
        for r, inj in enumerate(injections):
            S, Nr = inj["n_inj_steps"], inj["n_total"]
            j_max = min(Nr, int(math.ceil(n2 * Nr / S)) + 1) if S > 0 else Nr
            if j_max > injected[r]:
                sim.inject(inj, j_max - injected[r], inj.get("pid0", 0) + injected[r])
                injected[r] = j_max
        sim.step(n2 - n0)
        n0 = n2
    return n0


class Run:
    """One context on the workload plus its lazy continuous-injection plan."""

    def __init__(self, F, cfg, raw, precision, block, spl, compact, sort=1, load=True, tile=None, inj_every=None):
        import torch
        self.torch = torch
        self.cfg = cfg
        self.p = dict(cfg["params"], precision=precision)
        self.inj = cfg["injection"]
        self.N = int(cfg["n_particles"])
        self.S = int(self.inj["n_inj_steps"])
        self.sim = F.Simulation(self.p, cfg["grid"], self.N)
        torch.cuda.synchronize()
        t = time.time()
        if load:
            self.sim.load_grid(raw)
        self.load_s = time.time() - t
        self.sim.set_launch(block, spl, compact, sort)
        if tile is not None:
            self.sim.set_record_tile(tile)
        self.sim.set_timing(True)
        self.every = int(inj_every or spl)
        self.injected = [0]
        self.n0 = 0

    def reset(self):
        self.sim.reset()
        self.injected = [0]
        self.n0 = 0

    def chunk(self, n):
        """Step n global steps, the injection a launch (steps_per_launch, or
        inj_every) ahead (see advance)."""
        self.n0 = advance(self.sim, [dict(self.inj, n_total=self.N, n_inj_steps=self.S)], self.injected,
                          self.n0, self.n0 + n, self.every)

    def close(self):
        self.sim.close()


def timed(run, K, chunk, total=None):
    """K bench steps of `chunk` global steps each; with `total`, the last ones
    are cut so that the K steps take exactly `total` global steps."""
    torch = run.torch
    st0 = run.sim.stats()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.time()
    e0.record()
    done = 0
    for k in range(K):
        n = chunk if total is None else max(0, min(chunk, total - done))
        if n > 0:
            run.chunk(n)
        done += n
        if (k + 1) % max(1, K // 6) == 0:
            log(f"  chunk {k + 1}/{K} enqueued")
    e1.record()
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms = e0.elapsed_time(e1)
    st1 = run.sim.stats()
    steps = st1.particle_steps - st0.particle_steps
    kms = st1.step_kernel_ms - st0.step_kernel_ms
    nl = st1.step_launches - st0.step_launches
    return dict(ms=ms, wall=wall, particle_steps=int(steps), kernel_ms=kms, launches=int(nl), stats=st1,
                global_steps=done)


def graph_leg(run, K, chunk, total, j_direct):
    """The same run recorded as one launch graph (fte_capture_begin/end) and
    replayed from a reset: its time next to the direct calls', and the
    largest difference of the binned intensities."""
    torch = run.torch
    side = torch.cuda.Stream()
    torch.cuda.synchronize()
    with torch.cuda.stream(side):
        run.reset()
        t = time.time()
        run.sim.capture_begin()
        done = 0
        for k in range(K):
            n = max(0, min(chunk, total - done))
            if n > 0:
                run.chunk(n)
            done += n
        graph = run.sim.capture_end()
        build_s = time.time() - t
        run.reset()
        st0 = run.sim.stats()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        run.sim.graph_launch(graph)
        e1.record()
        side.synchronize()
        ms = e0.elapsed_time(e1)
        st1 = run.sim.stats()
        js, _ = run.sim.bin_observers()
        graph.close()
    steps = int(st1.particle_steps - st0.particle_steps)
    return dict(ms=round(ms, 1), particle_steps=steps, value=steps / (ms / 1e3), record_and_instantiate_s=round(build_s, 2),
                max_abs_diff_j_vs_direct=float(np.abs(js - j_direct).max()))


def gradient_leg(F, W, raw, args):
    """Differentiation workload (10^6 protons, 8,000 steps, smoothed
    intensities at the three 1-au observers): time of the plain forward pass,
    of the forward pass with smoothed sums, and of the gradient pass (tangents
    + derivative sums), each over the whole run.  Then the gradient of the
    summed intensity against central differences (h = 1e-3 and 1e-2, common
    random numbers) of the smoothed forward pass on the GPU, for several seeds, with
    the tangents' mu = 0 term of Eq. 5 (kink_sigma: a Gaussian of that width,
    or, negative, the bridge occupation of mu = 0) and without it: the mean
    over seeds of gradient minus difference, relative to the mean difference,
    with its standard error."""
    import torch
    cfg = W.cir_differentiation(precision=args.precision)
    n_steps = cfg["n_steps"]
    chunk = n_steps // 10
    p_grad = cfg["params"]
    if args.kink_sigma is not None:
        p_grad = dict(p_grad, kink_sigma=args.kink_sigma)
    if args.grad_dt_scale != 1.0:
        # the same physical run in steps scaled by grad_dt_scale (the
        # injection spread over the same time)
        s = args.grad_dt_scale
        n_steps = int(round(n_steps / s))
        chunk = n_steps // 10
        p_grad = dict(p_grad, dt=p_grad["dt"] * s)
        inj = dict(cfg["injection"], n_inj_steps=int(round(cfg["injection"]["n_inj_steps"] / s)))
        cfg = dict(cfg, n_steps=n_steps, injection=inj)
    p_smooth = dict(p_grad, grad=0)
    p_plain = {k: v for k, v in p_grad.items() if k not in ("smoothing", "grad", "kink_sigma")}

    def run(params, inj=None, timed_run=True):
        c = dict(cfg, params=params, injection=inj or cfg["injection"])
        r = Run(F, c, raw, args.precision, args.block, args.spl, args.compact, args.sort)
        res = timed(r, 10, chunk) if timed_run else None
        return r, res

    out = {"workload": cfg["name"], "particles": cfg["n_particles"], "global_steps": n_steps,
           "dt": p_grad["dt"], "kink_sigma": p_grad["kink_sigma"]}
    r, res = run(p_plain)
    r.close()
    # warm the other two modes once, untimed, then time them
    for params in (p_smooth, p_grad):
        r, _ = run(params, timed_run=False)
        r.chunk(chunk)
        torch.cuda.synchronize()
        r.close()
    r, res = run(p_plain)
    out["forward_ms"] = round(res["ms"], 2)
    out["forward_particle_steps"] = res["particle_steps"]
    r.close()
    r, res = run(p_smooth)
    out["forward_smoothed_ms"] = round(res["ms"], 2)
    r.close()
    r, res = run(p_grad)
    out["gradient_ms"] = round(res["ms"], 2)
    out["gradient_kernel_ms"] = round(res["kernel_ms"], 2)
    J, _ = r.sim.bin_smoothed()
    out["J_nonzero"] = int((J > 0).sum())
    r.close()
    out["grad_over_forward"] = round(out["gradient_ms"] / out["forward_ms"], 3)
    out["grad_over_smoothed_forward"] = round(out["gradient_ms"] / out["forward_smoothed_ms"], 3)

    def full(params, inj=None):
        rr, _ = run(params, inj=inj, timed_run=False)
        for _ in range(10):
            rr.chunk(chunk)
        return rr

    keys = ("lambda_ref", "kperp_ratio", "gamma_inj")
    steps_h = (1e-3, 1e-2)
    rows = {"kink": [], "bridge": [], "no_kink": []}
    fds = {h: [] for h in steps_h}
    for seed in range(args.grad_seeds):
        ps = dict(p_grad, seed=seed)
        for name, ks in (("kink", p_grad["kink_sigma"]), ("bridge", -1.0), ("no_kink", 0.0)):
            rr = full(dict(ps, kink_sigma=ks))
            Js, _ = rr.sim.bin_smoothed()
            rows[name].append(rr.sim.grad_of(np.ones(Js.shape)))
            rr.close()
        for h in steps_h:
            fd = []
            for key in keys:
                Jpm = []
                for sgn in (1, -1):
                    if key == "gamma_inj":
                        base = cfg["injection"]["gamma_inj"]
                        rr = full(dict(ps, grad=0), inj=dict(cfg["injection"], gamma_inj=base * (1 + sgn * h)))
                    else:
                        base = ps[key]
                        rr = full(dict(ps, grad=0, **{key: base * (1 + sgn * h)}))
                    Jpm.append(rr.sim.bin_smoothed()[0].sum())
                    rr.close()
                fd.append((Jpm[0] - Jpm[1]) / (2 * h * base))
            fds[h].append(np.array(fd))
        log(f"  gradient seed {seed}: kink {rows['kink'][-1]}, bridge {rows['bridge'][-1]}, "
            f"no kink {rows['no_kink'][-1]}, "
            f"fd {[list(fds[h][-1]) for h in steps_h]}")
    out["fd_seeds"] = args.grad_seeds
    for h in (steps_h if args.grad_seeds else ()):
        fd = np.array(fds[h])
        m = fd.mean(axis=0)
        tag = f"h{h:g}"
        out[f"fd_mean_{tag}"] = [float(v) for v in m]
        for name in ("kink", "bridge", "no_kink"):
            g = np.array(rows[name])
            d = g - fd
            # rel: mean over seeds of (gradient - difference) relative to the
            # mean difference; l1: sum |gradient - difference| / sum |difference|
            # over seeds (meaningful also where the seeds' differences change
            # sign); per_seed: each seed's relative deviation
            out[f"{name}_vs_fd_{tag}"] = {
                k: {"rel": float(d[:, q].mean() / m[q]),
                    "se": float(d[:, q].std(ddof=1) / math.sqrt(len(d)) / abs(m[q])) if len(d) > 1 else None,
                    "l1": float(np.abs(d[:, q]).sum() / np.abs(fd[:, q]).sum()),
                    "per_seed": [round(float(v), 4) for v in d[:, q] / fd[:, q]]}
                for q, k in enumerate(keys)}
    # control: the same workload and check with ISO scattering (D_mumu smooth
    # in mu, no mu = 0 term to carry).  The kappa ratio's derivative is small
    # and changes sign between seeds, so one seed's relative deviation says
    # little: the control keeps each seed's values and sums over seeds
    ctl = {f"h{h:g}": {k: {"grad": [], "fd": []} for k in keys[:2]} for h in steps_h}
    for seed in range(args.iso_seeds):
        pi = dict(p_grad, dmm_model="iso", seed=seed)
        rr = full(pi)
        Js, _ = rr.sim.bin_smoothed()
        gi = rr.sim.grad_of(np.ones(Js.shape))
        rr.close()
        for h in steps_h:
            for q, key in enumerate(keys[:2]):
                Jpm = []
                for sgn in (1, -1):
                    rr = full(dict(pi, grad=0, **{key: pi[key] * (1 + sgn * h)}))
                    Jpm.append(rr.sim.bin_smoothed()[0].sum())
                    rr.close()
                c = ctl[f"h{h:g}"][key]
                c["grad"].append(float(gi[q]))
                c["fd"].append(float((Jpm[0] - Jpm[1]) / (2 * h * pi[key])))
        log(f"  iso control seed {seed}: {ctl}")
    for tag in ctl:
        for c in ctl[tag].values():
            g, fd = np.array(c["grad"]), np.array(c["fd"])
            # rel: summed gradient minus summed difference over the summed
            # difference; l1: sum |gradient - difference| / sum |difference|
            c["rel"] = round(float((g - fd).sum() / fd.sum()), 4) if len(fd) else None
            c["l1"] = round(float(np.abs(g - fd).sum() / np.abs(fd).sum()), 4) if len(fd) else None
    out["iso_control"] = dict(ctl, seeds=args.iso_seeds)
    return out


def ensemble_leg(F, W, args):
    """Batched ensemble: 64 uneven runs (lambda, kappa ratio, particle and
    step counts drawn per run) as one population, autotuned, against the same
    runs stepped one context at a time with the default launch shape."""
    import torch
    dev = torch.device("cuda:0")
    cfg = W.cir_ensemble(precision=args.precision)
    g = cfg["grid"]
    raw = W.make_raw(g, cfg["wind"], xp=torch, device=dev)
    torch.cuda.synchronize()
    p = cfg["params"]
    N = cfg["n_particles"]
    out = {"workload": cfg["name"], "runs": len(cfg["runs"]), "particles": N,
           "max_steps": cfg["n_steps"], "snapshots": g["n_snap"], "leaves": int(len(g["leaves"]))}
    chunk = 640
    # one injection call per run per interval: a coarser interval than one
    # launch trades a few idle lanes for fewer launches of the 64 runs
    every = args.ens_inj_every

    def ensemble(tune):
        sim = F.Simulation(p, g, N)
        sim.load_grid(raw)
        sim.set_launch(args.block, args.spl, args.compact, args.sort)
        injected = [0] * len(cfg["injections"])
        best = None
        torch.cuda.synchronize()
        t_tune = 0.0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = 0.0
        n0 = 0
        while n0 < cfg["n_steps"]:
            n1 = min(n0 + chunk, cfg["n_steps"])
            if tune and best is None and n0 >= 2 * chunk:
                t = time.time()
                best = sim.autotune(4 * args.spl)
                t_tune = time.time() - t
            e0.record()
            advance(sim, cfg["injections"], injected, n0, n1, every)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            n0 = n1
        st = sim.stats()
        sim.close()
        return ms, int(st.particle_steps), best, t_tune

    ms, steps, best, t_tune = ensemble(True)
    out.update(ensemble_ms=round(ms, 1), particle_steps=steps, value=steps / (ms / 1e3),
               autotuned=dict(block=best[0], steps_per_launch=best[1], compact_every=best[2]) if best else None,
               autotune_s=round(t_tune, 2))
    ms0, steps0, _, _ = ensemble(False)
    out.update(ensemble_untuned_ms=round(ms0, 1))
    if best and not args.no_graph:
        # the whole ensemble at the tuned launch shape, its calls made
        # directly without a synchronisation between chunks, then recorded
        # as one launch graph and replayed from a reset
        def calls(sim):
            injected = [0] * len(cfg["injections"])
            n0 = 0
            while n0 < cfg["n_steps"]:
                n1 = min(n0 + chunk, cfg["n_steps"])
                advance(sim, cfg["injections"], injected, n0, n1, every)
                n0 = n1
        side = torch.cuda.Stream()
        torch.cuda.synchronize()
        with torch.cuda.stream(side):
            sim = F.Simulation(p, g, N)
            sim.load_grid(raw)
            sim.set_launch(best[0], best[1], best[2], args.sort)
            side.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            calls(sim)
            e1.record()
            side.synchronize()
            direct_ms = e0.elapsed_time(e1)
            direct_steps = int(sim.stats().particle_steps)
            sim.reset()
            t = time.time()
            sim.capture_begin()
            calls(sim)
            gr = sim.capture_end()
            build_s = time.time() - t
            sim.reset()
            e0.record()
            sim.graph_launch(gr)
            e1.record()
            side.synchronize()
            graph_ms = e0.elapsed_time(e1)
            graph_steps = int(sim.stats().particle_steps)
            gr.close()
            sim.close()
        out["graph"] = dict(direct_ms=round(direct_ms, 1), graph_ms=round(graph_ms, 1),
                            vs_direct=round(direct_ms / graph_ms, 4), record_and_instantiate_s=round(build_s, 2),
                            particle_steps_equal=direct_steps == graph_steps)
    # the same runs one context at a time (each loads the grid; not timed)
    seq_ms = 0.0
    seq_steps = 0
    for r, run in enumerate(cfg["runs"]):
        q = {k: v for k, v in p.items() if k != "runs"}
        q.update(run_id=p["run_id"] + r, lambda_ref=run["lambda_ref"], kperp_ratio=run["kperp_ratio"])
        inj = dict(cfg["injections"][r], run=0)
        c1 = dict(cfg, params=q, injection=inj, n_particles=inj["n_total"])
        rr = Run(F, c1, raw, args.precision, args.block, args.spl, args.compact, args.sort, inj_every=every)
        n_chunks = int(math.ceil(run["n_steps"] / chunk))
        ch = int(math.ceil(run["n_steps"] / n_chunks))
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        left = run["n_steps"]
        while left > 0:
            rr.chunk(min(ch, left))
            left -= min(ch, left)
        e1.record()
        torch.cuda.synchronize()
        seq_ms += e0.elapsed_time(e1)
        seq_steps += int(rr.sim.stats().particle_steps)
        rr.close()
    out.update(sequential_ms=round(seq_ms, 1), sequential_particle_steps=seq_steps,
               sequential_value=seq_steps / (seq_ms / 1e3), ensemble_speedup=round(seq_ms / ms, 3))
    del raw
    torch.cuda.empty_cache()
    return out


def largest_leg(F, W, args, hours=None):
    """The largest workload (shocked CIR with compression 3 at both shocks, 3
    AMR levels, 2,880 leaves, 96 hourly snapshots, kappa_perp, 10^8
    particles, 5 observers x 20 energies x 288 time bins) over its whole
    run (or its first `hours` of continuous injection): the step throughput
    and the memory it holds."""
    import torch
    dev = torch.device("cuda:0")
    c = W.cir_largest(precision=args.precision)
    g = c["grid"]
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()       # this leg's own peak below
    t = time.time()
    raw = W.make_raw(g, c["wind"], xp=torch, device=dev)
    torch.cuda.synchronize()
    wind_s = time.time() - t
    r = Run(F, c, raw, args.precision, args.block, args.spl, args.compact, args.sort)
    del raw
    torch.cuda.empty_cache()
    chunk = 576
    n_steps = c["n_steps"] if hours is None else min(c["n_steps"], int(hours * 3600 / c["params"]["dt"]))
    res = timed(r, -(-n_steps // chunk), chunk, total=n_steps)
    st = res["stats"]
    sz = F.fte_query_sizes(r.p, g, c["n_particles"])
    lv = np.asarray(g["leaves"])
    out = {"workload": c["name"], "leaves": int(len(lv)), "leaf_cells": int(len(lv) * np.prod(g["bx"])),
           "levels": 3, "snapshots": g["n_snap"], "particle_store": c["n_particles"],
           "global_steps": n_steps, "of_steps": c["n_steps"], "particles_injected": int(st.n_injected),
           "particle_steps": res["particle_steps"], "ms": round(res["ms"], 1),
           "value": res["particle_steps"] / (res["ms"] / 1e3), "grid_GB": round(sz.grid_bytes / 1e9, 2),
           "state_GB": round(2 * sz.state_bytes / 1e9, 2), "hist_MB": round(sz.hist_bytes / 1e6, 2),
           "wind_gen_s": round(wind_s, 2), "grid_load_s": round(r.load_s, 2),
           "device_peak_GB": round(torch.cuda.max_memory_allocated() / 1e9, 1),
           "retired": list(st.n_retired), "device_flags": int(st.device_flags)}
    r.close()
    del r
    torch.cuda.empty_cache()
    return out


def pool_leg(F, W, args, hours=12.0, wind_max=800e3):
    """The largest workload over its first `hours` with the grid held as a
    ring of 3 snapshot slots that each hold only the leaves the particles can
    reach (fte_plan_snapshot: the held particles and the injection shell,
    speeds up to 1.5 v_max + wind_max): per snapshot, the leaves the gather
    may read, the leaves held and the leaves whose input is copied into the
    load window (from device copies of the snapshot data standing in for
    the snapshot files); the record bytes against a ring of whole snapshots
    and the fully resident grid, and the input bytes copied against whole
    snapshots; the throughput with the planning, copies and loads in the
    timed region."""
    import torch
    dev = torch.device("cuda:0")
    c = W.cir_largest(precision=args.precision)
    g = c["grid"]
    p = dict(c["params"], precision=args.precision)
    inj = c["injection"]
    N, S = c["n_particles"], inj["n_inj_steps"]
    raw = W.make_raw(g, c["wind"], xp=torch, device=dev)     # stands in for the snapshot files
    nl = len(g["leaves"])
    cells = int(np.prod(g["bx"]))
    per = int(round(g["dt_s"] / p["dt"]))
    n_steps = min(c["n_steps"], int(hours * 3600 / p["dt"]))
    gs = dict(g, n_slots=3, n_pool=nl)
    sim = F.Simulation(p, gs, N)
    sim.set_launch(args.block, args.spl, args.compact, args.sort)
    sim.set_timing(True)
    stage = torch.empty((5,) + tuple(raw.shape[1:]), dtype=torch.float64, device=dev)
    counts, copied = [], 0
    injected = [0]

    def load(k):
        # copy only the input leaves of snapshots k-2 .. k+2 into the window
        leaves, cnt = sim.plan_snapshot(k, [inj], wind_max)
        counts.append(cnt)
        idx = torch.from_numpy(leaves.astype(np.int64)).to(dev)
        nonlocal copied
        for j in range(max(0, k - 2), min(g["n_snap"], k + 3)):
            stage[j - k + 2].index_copy_(0, idx, raw[j].index_select(0, idx))
            copied += len(leaves) * cells * 48
        ptrs = [stage[i].data_ptr() if 0 <= k - 2 + i < g["n_snap"] else 0 for i in range(5)]
        F.fte_load_snapshot(sim.ctx, k, ptrs, sim.stream)

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    load(0)
    load(1)
    done = 0
    while done < n_steps:
        k = done // per
        if k > 0 and done % per == 0 and k + 1 < g["n_snap"]:
            load(k + 1)
        done = advance(sim, [inj], injected, done, min((k + 1) * per, n_steps), args.spl)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = sim.stats()
    rec_ring_pool = F.fte_query_sizes(p, dict(gs, n_pool=max(cc[1] for cc in counts)), N).grid_bytes
    rec_ring_full = F.fte_query_sizes(p, dict(g, n_slots=3), N).grid_bytes
    rec_full = F.fte_query_sizes(p, g, N).grid_bytes
    sim.close()
    del stage, raw
    torch.cuda.empty_cache()
    frac = [round(cc[0] / nl, 3) for cc in counts]
    return dict(workload=c["name"], hours=hours, global_steps=n_steps, leaves=nl, snapshots_loaded=len(counts),
                gather_leaves_min_max=[min(cc[0] for cc in counts), max(cc[0] for cc in counts)],
                held_leaves_max=max(cc[1] for cc in counts), input_leaves_max=max(cc[2] for cc in counts),
                gather_fraction_per_snapshot=frac, device_flags=int(st.device_flags),
                record_bytes_pool_at_peak=int(rec_ring_pool), record_bytes_ring_whole=int(rec_ring_full),
                record_bytes_resident=int(rec_full), input_bytes_copied=int(copied),
                input_bytes_whole_snapshots=int(len(counts) * 5 * nl * cells * 48),
                particle_steps=int(st.particle_steps), ms=round(ms, 1),
                value=st.particle_steps / (ms / 1e3))


def paper_leg(F, W, args, levels=(1, 2, 3)):
    """The paper's own experiment (section 2.3) on the synthetic CIR in its
    corotating frame: a Green's-function run of 10^6 protons of 1 MeV injected
    where div V < 0, weight r^-2, for 36,000 steps of 10 s, at 1, 2 and 3 AMR
    levels; steady-state longitude profiles at 1.8 au, their peak per energy
    channel (the intensity-energy curves of the paper's AMR comparison) and the
    step throughput."""
    import torch
    dev = torch.device("cuda:0")
    out = {"workload": "paper_cir", "levels": {}}
    for nl in levels:
        c = W.paper_cir(n_levels=nl, precision=args.precision)
        g = c["grid"]
        raw = W.make_raw(g, c["wind"], xp=torch, device=dev)
        sim = F.Simulation(c["params"], g, c["n_particles"])
        sim.load_grid(raw)
        del raw
        sim.set_launch(args.block, args.spl, args.compact, args.sort)
        if args.tile_bytes is not None:
            sim.set_record_tile(args.tile_bytes)
        sim.inject(c["injection"], c["n_particles"], 0)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        left = c["n_steps"]
        while left > 0:
            k = min(3600, left)
            sim.step(k)
            left -= k
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        st = sim.stats()
        J, sig = sim.bin_steady()
        sim.close()
        del sim
        torch.cuda.empty_cache()
        J = J.reshape(len(c["ring_radii_au"]), -1, c["params"]["n_e"])
        e_lo = c["params"]["e_min"] * np.exp(np.arange(c["params"]["n_e"]) * c["params"]["dlne"]) / (1e3 * W.KEV)
        out["levels"][nl] = dict(leaves=int(len(g["leaves"])), particle_steps=int(st.particle_steps),
                                 value=st.particle_steps / (ms / 1e3), ms=round(ms, 1),
                                 peak_1p8au=[float("%.4g" % v) for v in J[-1].max(axis=0)])
    out["channel_lower_edges_MeV"] = [float("%.4g" % v) for v in e_lo]
    hi = [k for k in range(len(e_lo)) if e_lo[k] >= 1.99][:3]     # the channels from 2 MeV up
    base = out["levels"][levels[0]]["peak_1p8au"]
    out["gain_channels_MeV"] = [float("%.4g" % e_lo[k]) for k in hi]
    out["high_channel_gain_vs_level1"] = {nl: [round(out["levels"][nl]["peak_1p8au"][k] / base[k], 2) if base[k] else None
                                                for k in hi] for nl in levels}
    return out


def stream_leg(F, W, cfg, raw, args, total, n_slots=3, j_resident=None):
    """The CIR workload with the grid held as a ring of n_slots snapshots:
    each snapshot is copied from pinned host memory into a five-snapshot
    device staging window on a copy stream, one snapshot ahead of the clock,
    while the step kernels run; it is derived into its slot (on the stepping
    stream, after its copy's event) just before the clock needs it.  The
    `total` steps (those of the resident run it is compared with) are timed,
    transfers included, against the fully resident grid's value."""
    import torch
    dev = torch.device("cuda:0")
    g = dict(cfg["grid"], n_slots=n_slots)
    ns = g["n_snap"]
    host = torch.empty(raw.shape, dtype=torch.float64, pin_memory=True)
    host.copy_(raw)
    per_snap = raw[0].numel()
    # device staging ring: snapshot j in stage[j % 5]
    stage = torch.empty((5,) + tuple(raw.shape[1:]), dtype=torch.float64, device=dev)
    run = Run(F, dict(cfg, grid=g), None, args.precision, args.block, args.spl, args.compact, args.sort,
              load=False)
    sim = run.sim
    p = run.p
    main = torch.cuda.current_stream(dev)
    copier = torch.cuda.Stream(device=dev)           # default priority
    ready = {}                                       # snapshot -> event after its copy
    freed = {}                                       # staging slot -> event after its last reader

    def fetch(j):
        """Copy snapshot j into its staging slot on the copy stream, once the
        load that last read that slot has run."""
        if j >= ns or j in ready:
            return
        with torch.cuda.stream(copier):
            ev = freed.get(j % 5)
            if ev is not None:
                copier.wait_event(ev)
            stage[j % 5].copy_(host[j], non_blocking=True)
            e = torch.cuda.Event()
            e.record(copier)
            ready[j] = e

    nxt = [0]

    def load_through(k):
        while nxt[0] <= min(k, ns - 1):
            j0 = nxt[0]
            ptrs = []
            for j in range(j0 - 2, j0 + 3):
                if 0 <= j < ns:
                    fetch(j)
                    main.wait_event(ready[j])
                    ptrs.append(stage[j % 5].data_ptr())
                else:
                    ptrs.append(0)
            F.fte_load_snapshot(sim.ctx, j0, ptrs, sim.stream)
            # the load of j0 is the last reader of snapshot j0 - 2's slot,
            # which snapshot j0 + 3 takes next: prefetch it behind this load
            e = torch.cuda.Event()
            e.record(main)
            freed[(j0 - 2) % 5] = e
            fetch(j0 + 3)
            nxt[0] += 1

    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    steps_per_snap = int(round(g["dt_s"] / p["dt"]))
    done = 0
    while done < total:
        k = done // steps_per_snap
        load_through(k + 1)
        m = min((k + 1) * steps_per_snap, total) - done
        run.chunk(m)
        done += m
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    st = sim.stats()
    js, _ = sim.bin_observers()
    run.close()
    del host, stage, ready, freed
    # the same trajectories as the resident grid: the binned intensities
    # agree up to the summation order of the atomics
    dj = None
    if j_resident is not None:
        sc = max(float(np.abs(j_resident).max()), 1e-300)
        dj = float(np.abs(js - j_resident).max() / sc)
    return dict(slots=n_slots, snapshots=ns, ms=round(ms, 1), particle_steps=int(st.particle_steps),
                value=st.particle_steps / (ms / 1e3),
                grid_bytes_ring=int(F.fte_query_sizes(p, g, cfg["n_particles"]).grid_bytes),
                grid_bytes_full=int(F.fte_query_sizes(p, cfg["grid"], cfg["n_particles"]).grid_bytes),
                host_to_device_bytes_per_snapshot=per_snap * 8, max_abs_diff_j_vs_resident=dj)


def cpu_info():
    """Host CPU model and counts, for the CPU-baseline record."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), affinity=len(os.sched_getaffinity(0)))


def cpu_baseline(cfg, raw_gpu, samples):
    """The FP64 oracle, built -O3 -march=native on this host, on the first
    n_pids particles over the first n_steps steps of the workload, with the
    snapshots those steps touch copied to the host; one timing per
    (n_pids, n_steps, threads) sample."""
    import tempfile
    import oracle
    path = oracle.use_native_build(os.path.join(tempfile.mkdtemp(prefix="fte_oracle_"), "liboracle_native.so"))
    g = cfg["grid"]
    p = dict(cfg["params"], precision="fp64")
    n_max = max(s[1] for s in samples)
    t_last = p["t0"] + (n_max - 1) * p["dt"]
    k_hi = min(g["n_snap"] - 1, int(math.floor((t_last - g["t_s0"]) / g["dt_s"])) + 2)
    raw = raw_gpu[: k_hi + 1].cpu().numpy()
    # only the snapshots held are valid: the grid description keeps its full
    # snapshot count so the time derivative uses the run's own stencil
    G = oracle.Grid(g, raw, snap0=0)
    out = []
    for n_pids, n_steps, n_threads in samples:
        parts = oracle.inject(p, cfg["injection"], n_pids, cfg["injection"].get("pid0", 0))
        h = np.zeros(oracle.hist_size(p))
        t = time.time()
        steps = oracle.run(p, G, parts, 0, n_steps, h, n_threads)
        dt = time.time() - t
        out.append(dict(value=steps / dt, unit="particle-steps/s", cores=n_threads, kind="oracle",
                        sample=f"pids 0..{n_pids - 1} (the first injected) x global steps 0..{n_steps - 1} "
                               f"of the same workload, FP64, {steps} particle-steps in {dt:.1f} s",
                        build="gcc -O3 -march=native -ffp-contract=off -fopenmp (built on this host)"))
    os.remove(path)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--particles", type=int, default=10_000_000)
    ap.add_argument("--precision", default="mixed")
    ap.add_argument("--block", type=int, default=256)
    ap.add_argument("--spl", type=int, default=64)
    ap.add_argument("--compact", type=int, default=64)
    ap.add_argument("--sort", type=int, default=1)
    ap.add_argument("--tile-bytes", type=int, default=None, help="LDS record tile budget (default: the library's)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-grad", action="store_true", help="skip the differentiation workload")
    ap.add_argument("--grad-seeds", type=int, default=8, help="seeds of the gradient-vs-differences check")
    ap.add_argument("--ens-inj-every", type=int, default=256,
                    help="global steps between the ensemble's injection calls (a multiple of --spl keeps "
                         "every launch whole)")
    ap.add_argument("--iso-seeds", type=int, default=2,
                    help="seeds of the same check with ISO scattering (the control)")
    ap.add_argument("--grad-dt-scale", type=float, default=1.0,
                    help="step of the gradient leg relative to the workload's (same physical run)")
    ap.add_argument("--kink-sigma", type=float, default=None,
                    help="width of the Gaussian mu = 0 term of the gradient leg (default: the workload's)")
    ap.add_argument("--no-largest", action="store_true", help="skip the largest workload")
    ap.add_argument("--largest-hours", type=float, default=None,
                    help="hours of the largest workload to time (default: the whole 95 h run)")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble workload")
    ap.add_argument("--no-paper", action="store_true", help="skip the paper's CIR experiment at 1-3 AMR levels")
    ap.add_argument("--no-stream", action="store_true", help="skip the snapshot-streaming run of the CIR workload")
    ap.add_argument("--no-pool", action="store_true", help="skip the leaf-pool streaming run of the largest workload")
    ap.add_argument("--no-graph", action="store_true", help="skip the launch-graph replays (main run, ensemble)")
    ap.add_argument("--cpu-pids", type=int, default=4000)
    ap.add_argument("--cpu-pids-1", type=int, default=250, help="pids of the single-thread oracle sample")
    ap.add_argument("--cpu-steps", type=int, default=2800)
    ap.add_argument("--calib-copy", action="store_true", help="also run a 2 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU only; the multi-GPU sharding of the path is described, not run",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch
    import fte_workloads as W
    from paper_2404_12164_amd import fte as F

    dev = torch.device("cuda:0")
    cfg = W.cir_time_dependent(n_particles=args.particles, precision=args.precision)
    g = cfg["grid"]
    total_steps = cfg["n_steps"]
    # the K bench steps always cover the whole run
    K = max(1, args.steps)
    chunk = -(-total_steps // K)
    log(f"workload {cfg['name']}: {len(g['leaves'])} leaves, {g['n_snap']} snapshots, {args.particles} particles, "
        f"{total_steps} steps in {K} bench steps of <= {chunk}")

    t = time.time()
    raw = W.make_raw(g, cfg["wind"], xp=torch, device=dev)
    torch.cuda.synchronize()
    gen_s = time.time() - t
    log(f"wind generated on the GPU in {gen_s:.1f} s ({raw.numel() * 8 / 1e9:.1f} GB)")

    if args.calib_copy:
        # a plain streaming kernel of known traffic (reads 2 GiB, writes 2 GiB)
        # for scaling the FETCH_SIZE / WRITE_SIZE counters
        a = torch.ones(2 ** 28, dtype=torch.int64, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.bitwise_not(a, out=b)
        torch.cuda.synchronize()
        del a, b

    run = Run(F, cfg, raw, args.precision, args.block, args.spl, args.compact, args.sort, tile=args.tile_bytes)
    log(f"grid loaded in {run.load_s:.2f} s")
    if args.warmup > 0:
        timed(run, args.warmup, chunk, total=total_steps)
        torch.cuda.synchronize()
        run.reset()
    log("timed region")
    res = timed(run, K, chunk, total=total_steps)
    value = res["particle_steps"] / (res["ms"] / 1e3)
    js, _ = run.sim.bin_observers()
    st = res["stats"]
    grid_load_s = run.load_s
    graph = None
    if not args.no_graph:
        log("the same run recorded as one launch graph and replayed")
        graph = graph_leg(run, K, chunk, total_steps, js)
        graph["vs_direct"] = round(graph["value"] / value, 4)
    run.close()
    del run
    log(f"  {value:.4g} particle-steps/s over {res['global_steps']} global steps")

    # ---- rooflines of the step kernel, per launch, from the live event
    # timing of the launches and the committed counters (per particle-step)
    F_fields = 13 if (cfg["params"].get("kperp_ratio", 0) > 0 or cfg["params"].get("lambda_perp", 0) > 0) else 10
    T_s = 2 if g["n_snap"] >= 2 else 1
    s_f = 4 if args.precision == "mixed" else 8
    kern = ("k_step<float,false,0,false,true,false,false>" if args.precision == "mixed"
            else "k_step<double,false,0,false,true,false,false>")
    nl = max(res["launches"], 1)
    launch_s = res["kernel_ms"] / 1e3 / nl
    ps_launch = res["particle_steps"] / nl
    # the corner bytes the gather asks for (8 T_s F s_f, plus the state each
    # launch reads and writes once): mostly served by the LDS tile, L1 and L2
    b_step = 8 * T_s * F_fields * s_f + 2 * 64 / args.spl
    gathered = dict(unit="GB/s", bytes_per_particle_step=b_step, achieved=round(b_step * ps_launch / launch_s / 1e9, 1),
                    note="bytes the gather requests; served mostly on chip, not an HBM figure")
    ctr = read_counters("k_step_cir_counters.txt" if args.precision == "mixed" else "k_step_cir_fp64_counters.txt", kern)
    roof = dict(kernel=kern, launches=res["launches"], avg_launch_ms=round(launch_s * 1e3, 4),
                particle_steps_per_launch=round(ps_launch), gathered=gathered)
    VALU_PEAK = 256 * 4 * 2.4e9 / 4       # wave64 VALU instructions/s: 256 CUs x 4 SIMDs, 4 cycles each
    if ctr is not None:
        hbm = ctr["hbm_bytes_per_particle_step"] * ps_launch
        hbm_rate = hbm / launch_s / 1e9
        valu = ctr["valu_insts_per_particle_step"] * ps_launch / launch_s
        roof["hbm_measured"] = dict(unit="GB/s", achieved=round(hbm_rate, 1), peak=HBM_PEAK_GBS,
                                    frac=round(hbm_rate / HBM_PEAK_GBS, 4))
        roof["valu"] = dict(unit="wave64 VALU instructions/s", achieved=round(valu, 1), peak=VALU_PEAK,
                            frac=round(valu / VALU_PEAK, 4),
                            insts_per_particle_step=ctr["valu_insts_per_particle_step"])
        if "trans_insts_per_particle_step" in ctr:
            # transcendental instructions occupy the SIMD 4x as long
            busy = (ctr["valu_insts_per_particle_step"] + 3 * ctr["trans_insts_per_particle_step"]) * ps_launch / launch_s
            roof["valu"]["frac_trans_weighted"] = round(busy / VALU_PEAK, 4)
        # the binding roof: VALU issue when it is the larger fraction
        if roof["valu"]["frac"] >= roof["hbm_measured"]["frac"]:
            roof.update(bound="alu", achieved=roof["valu"]["achieved"], peak=VALU_PEAK,
                        unit=roof["valu"]["unit"], frac=roof["valu"]["frac"])
        else:
            roof.update(bound="hbm", achieved=round(hbm_rate, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=roof["hbm_measured"]["frac"])
        roof["traffic"] = round(hbm)
        roof["counters"] = "profiles/" + ("k_step_cir_counters.txt" if args.precision == "mixed"
                                          else "k_step_cir_fp64_counters.txt")
    else:
        roof.update(bound="hbm", achieved=None, peak=HBM_PEAK_GBS, unit="GB/s", frac=None, traffic=None,
                    note="no counters for the current kernel source")
    # the bandwidth a plain device copy reaches on this GPU, next to the
    # nominal peak: 4 GiB read + 4 GiB written per copy
    src = torch.empty(2 ** 29, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 5 * 2 * src.numel() * 8 / (c0.elapsed_time(c1) / 1e3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    roof["measured_copy_GBs"] = round(copy_gbs, 1)

    extra = {}
    if not args.no_stream:
        log("CIR workload with a 3-snapshot ring streamed from pinned host memory")
        extra["stream"] = stream_leg(F, W, cfg, raw, args, total_steps, j_resident=js)
        extra["stream"]["vs_resident"] = round(extra["stream"]["value"] / value, 3)

    if not args.no_fp64 and args.precision == "mixed":
        log("FP64 path on the same workload")
        r64 = Run(F, cfg, raw, "fp64", args.block, args.spl, args.compact, args.sort)
        res64 = timed(r64, K, chunk, total=total_steps)
        r64.close()
        del r64
        extra["fp64_value"] = res64["particle_steps"] / (res64["ms"] / 1e3)
        extra["mixed_over_fp64"] = round(value / extra["fp64_value"], 3)
        kern64 = "k_step<double,false,0,false,true,false,false>"
        c64 = read_counters("k_step_cir_fp64_counters.txt", kern64)
        if c64 is not None:
            nl64 = max(res64["launches"], 1)
            ls64 = res64["kernel_ms"] / 1e3 / nl64
            ps64 = res64["particle_steps"] / nl64
            v64 = c64["valu_insts_per_particle_step"] * ps64 / ls64
            h64 = c64["hbm_bytes_per_particle_step"] * ps64 / ls64 / 1e9
            extra["fp64_roofline"] = dict(kernel=kern64, avg_launch_ms=round(ls64 * 1e3, 4),
                                          valu_frac=round(v64 / VALU_PEAK, 4), hbm_frac=round(h64 / HBM_PEAK_GBS, 4),
                                          traffic=round(c64["hbm_bytes_per_particle_step"] * ps64))

    if not args.no_grad:
        log("differentiation workload: forward, smoothed forward, gradient, central differences")
        extra["gradient"] = gradient_leg(F, W, raw, args)

    if not args.no_ensemble:
        log("batched ensemble: 64 runs as one population vs one context at a time")
        extra["ensemble"] = ensemble_leg(F, W, args)

    if not args.no_paper:
        log("the paper's CIR experiment: region injection, Green's function, 1-3 AMR levels")
        extra["paper"] = paper_leg(F, W, args)

    if not args.no_largest:
        log("largest workload: shocked CIR, 3 levels, 96 snapshots, 10^8 particles")
        extra["largest"] = largest_leg(F, W, args, hours=args.largest_hours)

    if not args.no_pool:
        log("largest workload, first 12 h, ring of 3 slots holding only the reachable leaves")
        extra["pool"] = pool_leg(F, W, args)

    cpu = None
    if not args.no_cpu:
        info = cpu_info()
        n_all = min(16, info["affinity"])      # the host CPU share of one GPU
        log(f"oracle CPU baseline on 1 and {n_all} threads ({info['cpu_model']}, nproc {info['nproc']})")
        one, allc = cpu_baseline(cfg, raw, [(args.cpu_pids_1, args.cpu_steps, 1),
                                            (args.cpu_pids, args.cpu_steps, n_all)])
        cpu = dict(allc, single_thread=dict(value=one["value"], sample=one["sample"]), **info)

    out = {
        "metric": "pseudo-particle steps/s on 1 MI355X (mixed vs FP64); adjoint/forward cost",
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": res["ms"] / K,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if args.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": cfg["name"], "particles": args.particles, "global_steps": res["global_steps"],
                   "chunk": chunk, "snapshots": g["n_snap"], "leaves": int(len(g["leaves"])),
                   "levels": g["n_levels"], "precision": args.precision, "block": args.block,
                   "steps_per_launch": args.spl, "compact_every": args.compact, "spatial_sort": args.sort},
        "roofline": roof,
        "cpu_baseline": cpu,
        "particle_steps": res["particle_steps"],
        "wind_gen_s": round(gen_s, 2),
        "grid_load_s": round(grid_load_s, 2),
        "observer_counts_nonzero": int((js > 0).sum()),
        "retired": [int(v) for v in st.n_retired],
        "graph": graph,
    }
    out.update(extra)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
