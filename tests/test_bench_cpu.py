"""bench.py host logic: the one-GPU guard and the rule that committed counter
figures apply only to the kernel source and instance they were taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def _profile(tmp_path, sha, kernel):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "p.txt").write_text(f"# header: not a value\nkernel_source_sha256_16: {sha}\nkernel: {kernel}\n"
                             f"hbm_bytes_per_particle_step: 250.5\nvalu_insts_per_particle_step: 21.0\n")
    return d


@pytest.mark.parametrize("same_source,same_kernel", [(True, True), (True, False), (False, True)])
def test_counters_apply_only_to_their_kernel(tmp_path, monkeypatch, same_source, same_kernel):
    """Committed counter figures are per particle-step (so they apply to any
    number of bench steps) and only to the kernel source and instance they
    were taken on."""
    sha = "1234567890abcdef"
    k = "k_step<float,false,0,false,true,false,false>"
    _profile(tmp_path, sha, k)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha if same_source else "ffffffffffffffff")
    got = bench.read_counters("p.txt", k if same_kernel else "k_step<double,false,0,false,true,false,false>")
    if same_source and same_kernel:
        assert got["hbm_bytes_per_particle_step"] == 250.5 and got["valu_insts_per_particle_step"] == 21.0
    else:
        assert got is None


class _Recorder:
    """Stands in for a Simulation: records the inject and step calls."""

    def __init__(self):
        self.calls = []

    def inject(self, inj, n, first_pid):
        self.calls.append(("inject", n, first_pid))

    def step(self, n):
        self.calls.append(("step", n))


@pytest.mark.parametrize("chunks", [[564] * 5, [846, 846, 100], [5640], [1, 63, 64, 65, 700]])
def test_injection_keeps_pace_with_launches(chunks):
    """Continuous injection in the bench: every call steps at most up to the
    next multiple of steps_per_launch, and before it every pid whose first
    step (pid * S / N) falls before that call's end has been injected, in pid
    order, whatever chunks the caller asks for."""
    N, S, spl = 100_000, 16_920, 64
    r = object.__new__(bench.Run)
    r.sim, r.inj, r.N, r.S, r.every, r.injected, r.n0 = _Recorder(), {"pid0": 0}, N, S, spl, [0], 0
    for m in chunks:
        r.chunk(m)
    n0, injected = 0, 0
    for c in r.sim.calls:
        if c[0] == "inject":
            assert c[2] == injected and c[1] > 0
            injected += c[1]
            continue
        n1 = n0 + c[1]
        assert c[1] > 0 and (n1 - 1) // spl == n0 // spl       # within one launch window
        # every pid whose first step can fall before n1 is there, no more
        assert injected == min(N, -(-n1 * N // S) + 1)
        n0 = n1
    assert n0 == sum(chunks) and r.n0 == n0


def test_advance_paces_every_run():
    """Several runs (an ensemble): before each stretch of steps every run has
    injected exactly its pids whose first step can fall before the
    stretch's end, from its own first pid; a run injected all at once
    (n_inj_steps 0) is injected before the first stretch."""
    injs = [dict(n_total=1000, n_inj_steps=3000, pid0=0), dict(n_total=50, n_inj_steps=700, pid0=1000),
            dict(n_total=7, n_inj_steps=0, pid0=1050)]
    sim, injected, every = _Recorder(), [0, 0, 0], 256
    n0 = 0
    for n1 in (640, 1280, 1281, 3000):
        n0 = bench.advance(sim, injs, injected, n0, n1, every)
        assert n0 == n1
    done = [0, 0, 0]
    pos = 0
    for c in sim.calls:
        if c[0] == "inject":
            r = [q for q, inj in enumerate(injs) if inj["pid0"] <= c[2] < inj["pid0"] + inj["n_total"]][0]
            assert c[2] == injs[r]["pid0"] + done[r]
            done[r] += c[1]
            continue
        end = pos + c[1]
        assert (end - 1) // every == pos // every
        for r, inj in enumerate(injs):
            S, Nr = inj["n_inj_steps"], inj["n_total"]
            assert done[r] == (min(Nr, -(-end * Nr // S) + 1) if S else Nr)
        pos = end
    assert pos == 3000 and done == [1000, 50, 7] and injected == done
