"""Batched execution (many q-points x frequencies with uneven blocks in one
persistent launch), hipGraph replay and the tile autotuner."""
import sys

import numpy as np
import pytest
import torch

from gpu_common import assert_hermitian_exact, device_problem, need_gpu, oracle_chi0, rel_fro
from paper_2506_03477_amd import Context
from synth import workload

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def batch():
    need_gpu()
    wl = workload(3, nk=2)      # 32 q-points, npb 384, uneven nocc / nunocc per block
    probs = [device_problem(wl, q=q)[0] for q in range(wl.nq)]
    return wl, probs


@pytest.mark.parametrize("path", ["fp32", "bf16x3"])
def test_batched_32q_one_launch(batch, path):
    wl, probs = batch
    _say(f"batched {wl.nq} q-points {path}")
    ctx = Context(0)
    ctx.chi0_accumulate(probs, precision=path, delta_min=wl.delta_min)
    ctx.sync()
    worst = 0.0
    for q in (0, 7, 31):
        ref = oracle_chi0(wl, q=q)
        err = rel_fro(probs[q].chi0.cpu().numpy(), ref)
        worst = max(worst, err.max())
        assert_hermitian_exact(probs[q].chi0)
    _say(f"  worst rel err over sampled q: {worst:.3e}")
    # BF16x3 floor is ~4e-6 sqrt(npb / K) with K / npb ~ 35 here
    assert worst <= (1e-6 if path == "fp32" else 2e-6)
    ctx.close()


def test_batched_graph_and_autotune(batch):
    wl, probs = batch
    _say("batched graph replay + autotune")
    ctx = Context(0)
    ctx.chi0_accumulate(probs, precision="fp32")
    torch.cuda.synchronize()
    direct = [p.chi0.clone() for p in probs]
    for rep in range(3):
        for p in probs:
            p.chi0.zero_()
        ctx.chi0_accumulate(probs, precision="fp32", graph=True)
        torch.cuda.synchronize()
        _ = torch.randn(4096, device="cuda").sum()
        for p, d in zip(probs, direct):
            assert torch.equal(p.chi0, d), rep
    best, ms = ctx.autotune(probs, "fp32", reps=1)
    _say(f"  autotune fp32: best tile {best} ({ctx.tile_info('fp32', best)}), ms {ms}")
    assert 0 <= best < ctx.tile_count("fp32") and all(m > 0 for m in ms)
    assert ctx.get_tile("fp32") == best
    ctx.chi0_accumulate(probs, precision="fp32")
    ctx.sync()
    ref = oracle_chi0(wl, q=3)
    assert np.all(rel_fro(probs[3].chi0.cpu().numpy(), ref) <= 1e-6)
    ctx.close()


def test_bf16_default_tile_follows_size(batch):
    """With no tile fixed or tuned, BF16x3 picks its configuration per call
    from the padded tile area: at npb 384 the 256 x 128 tall tiles would be
    mostly padding, so a square tile of at most 128 is chosen; a fixed tile
    still wins, and both give the oracle's chi0."""
    wl, probs = batch
    _say("bf16x3 default tile at npb 384")
    ctx = Context(0)
    assert ctx.last_tile("bf16x3") == -1
    sub = probs[:4]
    ctx.chi0_accumulate(sub, precision="bf16x3", delta_min=wl.delta_min)
    ctx.sync()
    auto = ctx.last_tile("bf16x3")
    info = ctx.tile_info("bf16x3", auto)
    _say(f"  chosen tile {auto}: {info}")
    assert info["tile_p"] <= 128 and info["tile_q"] <= 128
    got_auto = sub[0].chi0.cpu().numpy()
    ctx.set_tile("bf16x3", 7)
    ctx.chi0_accumulate(sub, precision="bf16x3", delta_min=wl.delta_min)
    ctx.sync()
    assert ctx.last_tile("bf16x3") == 7
    ref = oracle_chi0(wl, q=0)
    e_auto, e_tall = rel_fro(got_auto, ref).max(), rel_fro(sub[0].chi0.cpu().numpy(), ref).max()
    _say(f"  rel err: chosen {e_auto:.3e}, tall {e_tall:.3e}")
    assert e_auto <= 2e-6 and e_tall <= 2e-6
    ctx.close()


@pytest.mark.parametrize("tile", [None, 7])
def test_bf16_graph_replay(batch, tile):
    """BF16x3 chi0 replayed from a hipGraph (pair weights, the pre-split pass
    when the tall tile runs, the rank-K kernel, the reduction): each replay,
    with eager work and synchronizations between them, equals the eager call
    bit for bit, in overwrite and in accumulate mode."""
    wl, probs = batch
    sub = probs[:6]
    _say(f"bf16x3 graph replay, tile {tile}")
    ctx = Context(0)
    if tile is not None:
        ctx.set_tile("bf16x3", tile)
    ctx.chi0_accumulate(sub, precision="bf16x3", delta_min=wl.delta_min)
    ctx.sync()
    direct = [p.chi0.clone() for p in sub]
    for rep in range(3):
        for p in sub:
            p.chi0.fill_(7.0)
        ctx.chi0_accumulate(sub, precision="bf16x3", delta_min=wl.delta_min, graph=True)
        ctx.sync()
        _ = torch.randn(4096, device="cuda").sum()
        torch.cuda.synchronize()
        for p, d in zip(sub, direct):
            assert torch.equal(p.chi0, d), rep
    for rep in range(2):
        for p, d in zip(sub, direct):
            p.chi0.copy_(d)
        ctx.chi0_accumulate(sub, precision="bf16x3", delta_min=wl.delta_min, accumulate=True,
                            graph=True)
        ctx.sync()
        _ = torch.randn(4096, device="cuda").sum()
        torch.cuda.synchronize()
        for p, d in zip(sub, direct):
            assert torch.equal(p.chi0, 2 * d), rep
    if tile is not None:
        assert ctx.last_tile("bf16x3") == tile
    ref = oracle_chi0(wl, q=0)
    assert rel_fro(direct[0].cpu().numpy(), ref).max() <= 2e-6
    ctx.close()
