"""bench.py host logic: the one-GPU guard and the rule that committed counter
figures apply only to the kernel source and run shape they were taken on."""
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


def _profile(tmp_path, sha, algo):
    d = tmp_path / "profiles"
    d.mkdir()
    (d / "p.txt").write_text(f"# header: not a value\nkernel_source_sha256_16: {sha}\n"
                             f"bench_algo_bytes_per_launch: {algo}\nhbm_bytes_per_launch: 1.5e10\n")
    return d


@pytest.mark.parametrize("same_source,algo,want", [(True, 1.0e11, 1.5e10), (True, 1.005e11, 1.5e10),
                                                   (True, 1.2e11, None), (False, 1.0e11, None)])
def test_counters_apply_only_to_their_run(tmp_path, monkeypatch, same_source, algo, want):
    sha = bench.kernel_source_hash() if same_source else "0000000000000000"
    _profile(tmp_path, sha, 1.0e11)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: sha if same_source else "ffffffffffffffff")
    assert bench.read_traffic("p.txt", algo) == want
