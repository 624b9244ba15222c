"""Validation and ordering through the C ABI on the GPU:

* pairs with D = eps_unocc - eps_occ <= 0 contribute nothing and make
  chi0_sync() return CHI0_EINVAL with their number (chi0_accumulate, its
  graph replay and the histogram route); the flag is cleared when reported;
* calls on two streams alternating over one handle give the results of the
  same calls on one stream, bit for bit (the handle orders its workspace);
* a partial-tile cap below a call's needs splits it into launches over
  problems and frequency ranges (same results within the path's
  tolerance), and a cap below one frequency's tiles returns CHI0_ENOMEM.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_common import device_problem, need_gpu, oracle_chi0, rel_fro
from paper_2506_03477_amd import Block, Context, Problem
from paper_2506_03477_amd._lib import CHI0_EINVAL, CHI0_ENOMEM, Chi0Error
from synth import workload

pytestmark = pytest.mark.gpu
ZT = {"fp64": "c128", "fp32": "c64", "bf16x3": "c64"}
TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-5}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    c = Context(0)
    yield c
    c.close()


def _sync_status(ctx):
    try:
        ctx.sync()
        return 0, ""
    except Chi0Error as e:
        return e.code, str(e)


def _planted(wl, path):
    """The workload's blocks with D <= 0 planted: block 0 has its occupied
    and unoccupied energies swapped (every pair D < 0), block 1 has one
    unoccupied energy equal to an occupied one (one D = 0 pair) and one
    below it.  Returns (device problem, host blocks for the oracle, count)."""
    prob, _, blks = device_problem(wl, ztype=ZT[path])
    host = []
    for k, (z, eo, eu, wk, blk) in enumerate(blks):
        eo_h, eu_h = eo.cpu().numpy().copy(), eu.cpu().numpy().copy()
        if k == 0:
            eo_h = np.full_like(eo_h, eu_h.max() + 0.25)
        elif k == 1:
            eu_h[0] = eo_h[0]
            eu_h[1] = eo_h[-1] - 0.125
        prob.blocks[k] = Block(z, torch.from_numpy(eo_h).cuda(), torch.from_numpy(eu_h).cuda(), wk)
        host.append((z.cpu().numpy(), eo_h, eu_h, wk))
    bad = sum(oracle.nonpositive_pairs(eo, eu) for _, eo, eu, _ in host)
    return prob, host, bad


@pytest.mark.parametrize("path", ["fp64", "fp32", "bf16x3"])
def test_nonpositive_pairs_reported(ctx, path):
    wl = workload(0, npb=96, nk=3, nocc=6, nunocc=40, ztype=ZT[path])
    prob, host, bad = _planted(wl, path)
    assert bad > 0
    with pytest.raises(oracle.InvalidPairs):
        oracle.chi0_ref(host, wl.npb, wl.omega, wl.delta_min)
    ref = oracle.chi0_ref(host, wl.npb, wl.omega, wl.delta_min, strict=False)
    for graph in (False, True, True):
        ctx.chi0_accumulate([prob], precision=path, graph=graph)
        code, msg = _sync_status(ctx)
        _say(f"{path} graph={graph}: sync -> {code} ({msg})")
        assert code == CHI0_EINVAL and f"{bad} pair(s)" in msg
        err = rel_fro(prob.chi0.cpu().numpy(), ref)
        assert np.all(err <= TOL[path]), err          # the valid pairs' chi0
    # reported once: the flag is cleared, and a valid call syncs clean
    assert _sync_status(ctx)[0] == 0
    good, _, _ = device_problem(wl, ztype=ZT[path])
    ctx.chi0_accumulate([good], precision=path)
    assert _sync_status(ctx)[0] == 0
    assert np.all(rel_fro(good.chi0.cpu().numpy(), oracle_chi0(wl, ztype=ZT[path])) <= TOL[path])


def test_nonpositive_pairs_histogram_route(ctx):
    from paper_2506_03477_amd import HistSpec
    wl = workload(0, npb=40, nk=3, nocc=4, nunocc=30, ztype="c128")
    prob, host, bad = _planted(wl, "fp64")
    edges = oracle.log_edges(1e-3, 1.05, 8.0)
    spec = HistSpec(edges=np.asarray(edges), sigma=0.0)
    ctx.chi0_hist_accumulate([prob], [spec], precision="fp64")
    code, msg = _sync_status(ctx)
    _say(f"histogram route: sync -> {code} ({msg})")
    assert code == CHI0_EINVAL and f"{bad} pair(s)" in msg
    good, _, _ = device_problem(wl)
    ctx.chi0_hist_accumulate([good], [spec], precision="fp64")
    assert _sync_status(ctx)[0] == 0


def test_two_streams_alternating_equal_one_stream(ctx):
    """Two q-points of the same shapes; chi0 (BF16x3 and FP64) and the
    inverse alternate between two streams on one handle, each stream only
    ordered after the other by the handle.  Every output equals the
    one-stream result bit for bit."""
    wl = workload(3, nq=2, npb=200, nk=4, ztype="c64")
    wl64 = workload(3, nq=2, npb=200, nk=4, ztype="c128")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()

    def run(streams):
        outs = []
        for path, w in (("bf16x3", wl), ("fp64", wl64)):
            probs = [device_problem(w, q=q)[0] for q in range(2)]
            vs = torch.from_numpy(w.vsqrt()).cuda()
            invs = [torch.empty_like(p.chi0) for p in probs]
            torch.cuda.synchronize()
            for q in range(2):
                ctx.chi0_accumulate([probs[q]], precision=path, stream=streams[q])
            for q in range(2):
                ctx.dielectric_invert(vs, probs[q].chi0, invs[q], method="hpd", stream=streams[q])
            torch.cuda.synchronize()
            ctx.sync()
            outs += [p.chi0.cpu() for p in probs] + [x.cpu() for x in invs]
        return outs

    one = run([s1, s1])
    two = run([s1, s2])
    for a, b in zip(one, two):
        assert torch.equal(a, b)


@pytest.mark.parametrize("path", ["fp64", "bf16x3"])
def test_partial_cap_splits_launches(ctx, path):
    """Three problems x 4 frequencies at npb 300 under a cap that holds
    only about one problem-frequency of partial tiles: the call runs as many
    launches (frequency ranges and problems), with the same results."""
    w = workload(3, nq=3, npb=300, nk=3, omega=(0.0, 0.3, 1.1, 4.0), ztype=ZT[path])
    probs = [device_problem(w, q=q)[0] for q in range(3)]
    ctx.chi0_accumulate(probs, precision=path)
    ctx.sync()
    full = [p.chi0.clone() for p in probs]
    tile = ctx.last_tile(path)
    info = ctx.tile_info(path, tile)
    tp, tq = info["tile_p"], info["tile_q"]
    ntiles = sum(1 for a in range((300 + tp - 1) // tp)
                 for b in range((300 + tq - 1) // tq) if b * tq <= min((a + 1) * tp, 300) - 1)
    one = ntiles * tp * tq * 16
    try:
        ctx.set_tile(path, tile)                  # same kernel under the cap
        ctx.set_partial_cap(int(1.5 * one))
        for p in probs:
            p.chi0.fill_(7.0)
        ctx.chi0_accumulate(probs, precision=path)
        ctx.sync()
        for q, p in enumerate(probs):
            ref = oracle_chi0(w, q=q)
            e_cap = rel_fro(p.chi0.cpu().numpy(), ref)
            e_full = rel_fro(full[q].cpu().numpy(), ref)
            _say(f"{path} q={q}: capped {e_cap.max():.3e}, one launch {e_full.max():.3e}")
            assert np.all(e_cap <= TOL[path]) and np.all(e_full <= TOL[path])
        ctx.set_partial_cap(one // 2)             # one frequency does not fit
        with pytest.raises(Chi0Error) as ei:
            ctx.chi0_accumulate(probs, precision=path)
        assert ei.value.code == CHI0_ENOMEM
    finally:
        ctx.set_partial_cap(0)
        ctx.set_tile(path, -1)
    ctx.sync()


_LOG_SCRIPT = """
import sys, torch
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
from gpu_common import device_problem
from paper_2506_03477_amd import Context
from synth import workload
ctx = Context(0)
wl = workload(0)
prob, vsqrt, _ = device_problem(wl, ztype="c128")
ctx.chi0_accumulate([prob], precision="fp64")
inv = torch.empty_like(prob.chi0)
ctx.dielectric_invert(vsqrt, prob.chi0, inv, method="hpd")
ctx.sync()
ctx.close()
"""


@pytest.mark.parametrize("value", ["1", "0"])
def test_chi0_log_switch(value):
    """CHI0_LOG describes each launch on stderr (a child process, since the
    switch is read once per process); "0" keeps the library silent."""
    import os
    import subprocess
    need_gpu()
    tests = os.path.dirname(os.path.abspath(__file__))
    root = os.path.dirname(tests)
    env = dict(os.environ, CHI0_LOG=value)
    r = subprocess.run([sys.executable, "-c", _LOG_SCRIPT.format(root=root, tests=tests)],
                       env=env, capture_output=True, text=True, timeout=240)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stderr.splitlines() if l.startswith("[libchi0]")]
    if value == "1":
        assert any("rank-K launch: kind 0" in l for l in lines), r.stderr[-2000:]
        assert any("inverse: npb 64, 4 frequencies, method 1" in l for l in lines), r.stderr[-2000:]
    else:
        assert lines == []
