"""Host-side logic of bench.py (CPU): the one-GPU contract, the flop counts
against explicit counts on small sizes, the tile count against brute force,
the step's inverse choices against the binding, and the rule that stored
traffic counters count only for the kernel code they were taken on."""
import glob
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402
from paper_2506_03477_amd import _lib  # noqa: E402


@pytest.mark.parametrize("n", [2, 8])
def test_more_than_one_gpu_exits(n):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", str(n)],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


@pytest.mark.parametrize("npb,npairs,nomega", [(1, 1, 1), (3, 5, 2), (7, 2, 3)])
def test_zherk_flops_explicit(npb, npairs, nomega):
    # one complex multiply-add (8 real flops) per pair, per lower-triangle
    # entry (diagonal included), per frequency
    macs = sum(1 for _ in range(nomega) for _ in range(npairs)
               for p in range(npb) for q in range(npb) if p >= q)
    assert bench.zherk_flops(npb, npairs, nomega) == 8 * macs


@pytest.mark.parametrize("npb", [1, 5, 64, 100, 128, 257, 300])
@pytest.mark.parametrize("tp,tq", [(128, 128), (256, 128), (64, 64), (32, 16)])
def test_lower_tile_count_brute(npb, tp, tq):
    brute = 0
    for r in range(-(-npb // tp)):
        for c in range(-(-npb // tq)):
            rows = range(r * tp, min((r + 1) * tp, npb))
            cols = range(c * tq, min((c + 1) * tq, npb))
            if any(i >= j for i in rows for j in cols):
                brute += 1
    assert bench.lower_tile_count(npb, tp, tq) == brute


def test_step_inverse_choices_match_binding():
    assert set(bench.STEP_INVERSE) == set(_lib.INV_METHOD)


def test_source_sha_ignores_comments(tmp_path, monkeypatch):
    a = tmp_path / "a.hip"
    a.write_text("int f() { return 1; }  // note\n/* block\n comment */\n")
    monkeypatch.setitem(bench.KERNEL_SOURCE, "probe", (str(a),))
    s0 = bench.source_sha("probe")
    a.write_text("// other note\nint  f()  {\n return 1; }\n")
    assert bench.source_sha("probe") == s0
    a.write_text("int f() { return 2; }\n")
    assert bench.source_sha("probe") != s0


def test_stored_traffic_only_for_current_kernel(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("__global__ void k() {}\n")
    monkeypatch.setitem(bench.KERNEL_SOURCE, "probe", (str(src),))
    tf = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "traffic_file", lambda prec, name: str(tf))
    assert bench.stored_traffic("probe", "w") is None                   # no counters stored
    tf.write_text(json.dumps({"kernel_source_sha": bench.source_sha("probe"),
                              "traffic_bytes_per_launch": 1234.4}))
    assert bench.stored_traffic("probe", "w") == 1234
    src.write_text("// a comment only\n__global__ void k() {}\n")
    assert bench.stored_traffic("probe", "w") == 1234                   # comment edits keep them
    src.write_text("__global__ void k() { int x = 0; }\n")
    assert bench.stored_traffic("probe", "w") is None                   # code edits void them


def test_committed_traffic_files_well_formed():
    files = glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json"))
    assert files
    for f in files:
        with open(f) as fh:
            t = json.load(fh)
        assert len(t["kernel_source_sha"]) == 16 and t["traffic_bytes_per_launch"] > 0, f


@pytest.mark.parametrize("per_state,warm,nmax,tuple_out,fixed", [
    (0.5, 3.0, 1000, False, 0.0),      # a slow first call must not shrink the sample
    (0.5, 0.0, 1000, True, 0.0),
    (0.5, 0.0, 10, False, 0.0),        # capped by the states there are
    (100.0, 0.0, 1000, False, 0.0),    # one state already exceeds the target
    (0.04, 0.0, 200, True, 2.5),       # a fixed cost per call dominates small samples
    (0.7, 0.0, 1000, False, 6.0),
    (0.2, -1.0, 200, True, 0.0),       # the probe itself slowed (to 3 s) by noise
])
def test_size_sample(per_state, warm, nmax, tuple_out, fixed):
    calls = []

    def run(n):
        if warm < 0:                   # noise on the first two calls
            t = (3.0 if len(calls) < 2 else 0.0) + fixed + per_state * n
            calls.append(n)
            return (t, 7 * n) if tuple_out else t
        t = (warm if not calls else 0.0) + fixed + per_state * n
        calls.append(n)
        return (t, 7 * n) if tuple_out else t

    n, r = bench.size_sample(run, nmax, target_s=15.0)
    t = r[0] if tuple_out else r
    assert 1 <= n <= nmax and calls[-1] == n
    if tuple_out:
        assert r[1] == 7 * n
    if fixed + per_state * nmax >= 10.0 and fixed + per_state <= 15.0:
        assert 10.0 <= t <= 30.0, (n, t)
    assert sum(fixed + per_state * c for c in calls) <= 4 * 15.0 + per_state * 2
