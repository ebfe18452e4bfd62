"""Host-side logic of the benchmark (no GPU): the one-GPU guard, the rule
that a measured HBM traffic figure is dropped once its kernel's source has
changed, and the subdomain sizes behind the algorithmic byte counts, checked
against the oracle's decomposition (Sec. 3: overlapping blocks of the grid)."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from oracle import decomp, problem  # noqa: E402


def test_bench_refuses_several_gpus():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert p.returncode == 2, (p.returncode, p.stderr)
    assert "one GPU" in p.stderr and p.stdout == ""


def test_measured_traffic_follows_the_kernel_source(tmp_path, monkeypatch):
    committed = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))
    key, rec = next(iter(committed["kernels"].items()))
    src = tmp_path / rec["source"]
    src.parent.mkdir(parents=True)
    src.write_bytes(b"kernel source, first version")
    rec = dict(rec, sha256=hashlib.sha256(b"kernel source, first version").hexdigest(), traffic_bytes=123.0)
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "pmc_traffic.json").write_text(json.dumps({"kernels": {key: rec}}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic(key) == 123.0
    assert bench.measured_traffic("no_such_kernel") is None
    src.write_bytes(b"kernel source, second version")
    assert bench.measured_traffic(key) is None


@pytest.mark.parametrize("n,nsub,overlap", [(1025, 16, 2), (513, 10, 2), (385, 8, 2), (257, 6, 2),
                                            (193, 5, 2), (129, 4, 2), (65, 4, 1)])
def test_subdomain_sizes_match_the_oracle_decomposition(n, nsub, overlap):
    subs = decomp.decompose(n, problem.SOMMERFELD, nsub, nsub, overlap)
    assert bench.subdomain_sizes(n, nsub, overlap) == [(s.nx, s.ny) for s in subs]


def test_local_solve_bytes_count_every_inverse_block_twice():
    """Each Schur inverse G_j (nx^2 entries per grid line) is read by the
    forward and the backward sweep; the right-hand side is gathered in
    complex128 and the local solution written in the working precision."""
    subs = decomp.decompose(1025, problem.SOMMERFELD, 16, 16, 2)
    for s_bytes in (8, 16):
        want = sum(2 * s.ny * s.nx * s.nx * s_bytes + s.idx.size * (16 + s_bytes) for s in subs)
        assert bench.local_solve_bytes(bench.subdomain_sizes(1025, 16, 2), s_bytes) == want
    assert abs(bench.local_solve_bytes(bench.subdomain_sizes(1025, 16, 2), 8) - 1.3056e9) < 1e6


def test_nd_launch_plan_covers_every_level_once_per_direction():
    """The coarse solve's launches at n = 1025 (coarse grid 513 x 513), in
    dispatch order: the forward subtree launch (depths 8-12), the forward
    levels 7..1, the backward levels 0..7, the backward subtree launch; every
    level is covered once per direction (the root's forward part is done by
    its backward launch)."""
    import paper_2408_03571_amd as hs
    levels = hs.hs_nd_plan_level_stats(513, 513, 2)
    plan = bench.nd_launch_plan(levels)
    assert bench.nd_subtree_depth(levels) == 8 and len(plan) == bench.nd_launches(levels) == 17
    assert plan[0] == ("forward", [8, 9, 10, 11, 12]) and plan[-1] == ("backward", [8, 9, 10, 11, 12])
    fwd = sorted(lv for d, lvs in plan if d == "forward" for lv in lvs)
    bwd = sorted(lv for d, lvs in plan if d == "backward" for lv in lvs)
    assert fwd == list(range(1, 13)) and bwd == list(range(13))
    # a plan with no subtree levels is all level launches
    flat = [dict(s, subtree_workgroups=0) for s in levels]
    assert bench.nd_launches(flat) == 2 * len(levels) - 1
