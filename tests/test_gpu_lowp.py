"""GPU parity of the reduced-precision paths (FP32 and BF16x3 split products,
FP32 runs flushed into FP64) against the FP64 oracle at 1e-6 relative
Frobenius error per frequency, and against a numpy model of the split
arithmetic (which isolates kernel mistakes from the split's own error)."""
import sys
import time

import numpy as np
import pytest
import torch

import oracle
from gpu_common import (assert_hermitian_exact, device_problem, need_gpu, oracle_chi0,
                        rel_fro)
from paper_2506_03477_amd import Block, Context, Problem
from splitmodel import chi0_model
from synth import workload

pytestmark = pytest.mark.gpu
TOL = 1e-6


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    c = Context(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _model(wl, path, lolo=False):
    blocks = []
    for blk in wl.blocks(0):
        eo, eu = wl.energies(blk)
        blocks.append((wl.z_block(blk), eo, eu, blk.wk))
    return chi0_model(blocks, wl.npb, wl.omega, wl.delta_min, path, lolo)


# The BF16x3 split represents each operand to 16 significant bits, so its
# error relative to the oracle is about 4e-6 sqrt(npb / K) (K = number of
# pairs): the cases keep K / npb >= 200, as in the workloads themselves
# (K / npb = 1500 for npb = 2048).  FP32 has no such floor.
CASES = {
    "bf16x3": [
        (0, dict(ztype="c64", nk=64)),                            # npb 64 shape, 64 k-points
        (1, dict(npb=200, nk=4, ztype="c64")),                    # ragged npb, several tiles
        (2, dict(npb=160, nk=2, nocc=40, nunocc=500)),            # npb 2048 workload generator
        (3, dict(nq=1, npb=130, nk=16)),                          # uneven blocks
        (4, dict(npb=96, nk=4)),                                  # spins, intraband cut
    ],
    "fp32": [
        (0, dict(ztype="c64")),
        (1, dict(npb=200, nk=3, nocc=7, nunocc=45, ztype="c64")),
        (2, dict(npb=300, nk=2, nocc=9, nunocc=120)),
        (3, dict(nq=1, npb=130, nk=6)),
        (4, dict(npb=96, nk=3)),
    ],
}


@pytest.mark.parametrize("path,cfg,over", [(p, c, o) for p in CASES for c, o in CASES[p]])
def test_lowp_parity(ctx, path, cfg, over):
    wl = workload(cfg, **over)
    _say(f"{path} parity {wl.name} {over}")
    prob, _, _ = device_problem(wl)
    ctx.chi0_accumulate([prob], precision=path, delta_min=wl.delta_min)
    ctx.sync()
    got = prob.chi0.cpu().numpy()
    ref = oracle_chi0(wl)
    err = rel_fro(got, ref)
    mod = _model(wl, path)
    err_model = rel_fro(got, mod)
    _say(f"  vs oracle {err.max():.3e}  vs split model {err_model.max():.3e}  "
         f"model vs oracle {rel_fro(mod, ref).max():.3e}")
    assert np.all(err <= TOL), err
    assert np.all(err_model <= 3e-7), err_model
    assert_hermitian_exact(prob.chi0)


def test_bf16_lolo_and_flush_lengths(ctx):
    wl = workload(2, npb=160, nk=2, nocc=40, nunocc=500)
    _say("bf16x3 lolo / flush lengths")
    ref = oracle_chi0(wl)
    prob, _, _ = device_problem(wl)
    ctx.chi0_accumulate([prob], precision="bf16x3", lolo=True)
    ctx.sync()
    e_lolo = rel_fro(prob.chi0.cpu().numpy(), ref)
    assert np.all(e_lolo <= TOL)
    assert np.all(rel_fro(prob.chi0.cpu().numpy(), _model(wl, "bf16x3", lolo=True)) <= 3e-7)
    outs = []
    for fl in (16, 256, 0):
        ctx.set_flush(fl)
        ctx.chi0_accumulate([prob], precision="bf16x3")
        ctx.sync()
        outs.append(prob.chi0.clone())
        e = rel_fro(prob.chi0.cpu().numpy(), ref)
        _say(f"  flush {fl}: {e.max():.3e} (lolo {e_lolo.max():.3e})")
        assert np.all(e <= TOL)
    ctx.set_flush(0)
    assert not torch.equal(outs[0], outs[2])   # the flush length changes the rounding


def test_lowp_deterministic_graph_accumulate(ctx):
    wl = workload(3, nq=1, npb=200, nk=16)
    _say("bf16x3 determinism / graph / accumulate")
    prob, _, _ = device_problem(wl)
    ctx.chi0_accumulate([prob], precision="bf16x3")
    first = prob.chi0.clone()
    ctx.chi0_accumulate([prob], precision="bf16x3")
    torch.cuda.synchronize()
    assert torch.equal(first, prob.chi0)
    for rep in range(3):
        prob.chi0.zero_()
        ctx.chi0_accumulate([prob], precision="bf16x3", graph=True)
        torch.cuda.synchronize()
        _ = torch.randn(4096, device="cuda").sum()
        assert torch.equal(prob.chi0, first), rep
    prob.chi0.copy_(first)
    ctx.chi0_accumulate([prob], precision="bf16x3", accumulate=True)
    ctx.sync()
    assert np.all(rel_fro(prob.chi0.cpu().numpy(), 2 * first.cpu().numpy()) <= 1e-15)
    assert_hermitian_exact(prob.chi0)


@pytest.mark.parametrize("path", ["bf16x3", "fp32"])
def test_every_tile_configuration(ctx, path):
    """Every kernel variant of the autotuner's table meets the same bar (a
    ragged npb spanning several tiles of either size, uneven blocks)."""
    wl = workload(3, nq=1, npb=200, nk=16)
    ref = oracle_chi0(wl)
    mod = _model(wl, path)
    prob, _, _ = device_problem(wl)
    outs = []
    for tile in range(ctx.tile_count(path)):
        ctx.set_tile(path, tile)
        _say(f"{path} tile {tile} {ctx.tile_info(path, tile)}")
        ctx.chi0_accumulate([prob], precision=path)
        ctx.sync()
        got = prob.chi0.cpu().numpy()
        e, em = rel_fro(got, ref), rel_fro(got, mod)
        _say(f"  vs oracle {e.max():.3e}  vs split model {em.max():.3e}")
        assert np.all(e <= TOL), e
        assert np.all(em <= 3e-7), em
        assert_hermitian_exact(prob.chi0)
        outs.append(prob.chi0.clone())
    ctx.set_tile(path, -1)
    _say("  bitwise equal to tile 0: " + str([bool(torch.equal(outs[0], o)) for o in outs]))


def test_xcd_lockstep_bounded_and_neutral(ctx):
    """The XCD lockstep of the default BF16x3 kernel changes timing only:
    its output is bitwise the same with the lockstep off, at its default
    slack, at a slack of one stage, and with every wait made unmeetable
    (each workgroup then waits the full bound once and runs on without the
    lockstep, so the launch still ends within a bounded time)."""
    wl = workload(2, npb=256, nk=4)          # one problem of equal blocks: round-robin units
    prob, _, _ = device_problem(wl)
    ctx.set_tile("bf16x3", ctx.get_tile("bf16x3"))
    outs, secs = {}, {}
    for slack in (-1, 0, 1, -2, -1):
        ctx.set_xcd_slack(slack)
        t0 = time.perf_counter()
        ctx.chi0_accumulate([prob], precision="bf16x3", delta_min=wl.delta_min)
        ctx.sync()
        secs[slack] = time.perf_counter() - t0
        outs.setdefault(slack, prob.chi0.clone())
        assert torch.equal(prob.chi0, outs[-1]), slack
    ctx.set_xcd_slack(-1)
    ctx.set_tile("bf16x3", -1)
    _say("lockstep slack -> seconds: " + ", ".join(f"{k}: {v:.3f}" for k, v in secs.items()))
    assert secs[-2] < 30.0
    with pytest.raises(Exception):
        ctx.set_xcd_slack(-3)


@pytest.mark.parametrize("npb,omega", [(131, (0.0, 0.1, 0.5, 2.0, 8.0)),     # odd npb, 5 frequencies
                                       (256, (0.3, 3.0)),                     # group of two
                                       (200, tuple(np.geomspace(0.01, 100.0, 9)))])
def test_frequency_group_tile(ctx, npb, omega):
    """The frequency-group kernel (four frequencies of a tile per workgroup,
    operands staged once in LDS) on frequency counts that leave partial
    groups, odd npb and several tiles: against the oracle and the split
    model, equal to the per-wave kernel's result up to FP32 rounding, and
    bitwise equal across its variants (hints, atomic flushes, load
    timing)."""
    wl = workload(3, nq=1, npb=npb, nk=16, omega=omega)
    ref = oracle_chi0(wl)
    mod = _model(wl, "bf16x3")
    prob, _, _ = device_problem(wl)
    grp = 13                                  # the frequency-group configuration
    info = ctx.tile_info("bf16x3", grp)
    assert (info["tile_p"], info["tile_q"], ctx.tile_lists("bf16x3", grp)) == (128, 64, 1)
    got = {}
    for tile in (grp, 14, 15, 16, 17, 18, 19, 20, 11):
        ctx.set_tile("bf16x3", tile)
        ctx.chi0_accumulate([prob], precision="bf16x3")
        ctx.sync()
        got[tile] = prob.chi0.cpu().numpy()
        assert_hermitian_exact(prob.chi0)
    # tile 20 reads Z in 16-byte chunks (even npb): the same values two
    # complex64 elements into a larger allocation (16-byte aligned, not
    # cache-line aligned) give the same bits
    shifted = []
    for b in prob.blocks:
        buf = torch.empty(b.z.numel() + 2, dtype=b.z.dtype, device=b.z.device)
        zz = buf[2:].view(b.z.shape)
        zz.copy_(b.z)
        assert zz.data_ptr() % 128 == 16
        shifted.append(Block(zz, b.eps_occ, b.eps_unocc, b.wk))
    prob16 = Problem(shifted, prob.omega, torch.empty_like(prob.chi0))
    ctx.set_tile("bf16x3", 20)
    ctx.chi0_accumulate([prob16], precision="bf16x3")
    ctx.sync()
    got["20/16"] = prob16.chi0.cpu().numpy()
    ctx.set_tile("bf16x3", -1)
    e, em = rel_fro(got[grp], ref), rel_fro(got[grp], mod)
    _say(f"frequency groups npb {npb}, {len(omega)} omega: vs oracle {e.max():.3e}, "
         f"vs split model {em.max():.3e}, vs tile 11 {rel_fro(got[grp], got[11]).max():.3e}")
    assert np.all(e <= TOL), e
    assert np.all(em <= 3e-7), em
    assert np.all(rel_fro(got[grp], got[11]) <= 3e-7)
    # the issue-order hints, the atomic flushes (one wave per partial slot,
    # its additions in program order), the blocks left out above the
    # diagonal, the XCD lockstep, the planar partial tiles and the 16-byte
    # Z loads (odd npb: dword loads) change no arithmetic
    for t in (14, 15, 16, 17, 18, 19, 20, "20/16"):
        assert np.array_equal(got[t], got[grp]), t


@pytest.mark.parametrize("npb,omega", [(131, (0.0, 0.1, 0.5, 2.0, 8.0)),     # odd npb, 5 frequencies
                                       (256, (0.3, 3.0)),                     # group of two
                                       (200, tuple(np.geomspace(0.01, 100.0, 9)))])
def test_fp32_frequency_group_tile(ctx, npb, omega):
    """The FP32 frequency-group kernel on partial frequency groups, odd npb
    and several tiles: against the oracle and the exact-product model, and
    close to the 64^2 FP32 kernel (the FP32 sums differ in order only)."""
    wl = workload(3, nq=1, npb=npb, nk=16, omega=omega)
    ref = oracle_chi0(wl)
    mod = _model(wl, "fp32")
    prob, _, _ = device_problem(wl)
    grp = 2                                   # the FP32 frequency-group configuration
    info = ctx.tile_info("fp32", grp)
    assert (info["tile_p"], info["tile_q"]) == (128, 64) and ctx.tile_diag_skip("fp32", grp)
    got = {}
    for tile in (grp, 1):
        ctx.set_tile("fp32", tile)
        ctx.chi0_accumulate([prob], precision="fp32")
        ctx.sync()
        got[tile] = prob.chi0.cpu().numpy()
        assert_hermitian_exact(prob.chi0)
    ctx.set_tile("fp32", -1)
    e, em = rel_fro(got[grp], ref), rel_fro(got[grp], mod)
    _say(f"fp32 frequency groups npb {npb}, {len(omega)} omega: vs oracle {e.max():.3e}, "
         f"vs exact-product model {em.max():.3e}, vs tile 1 {rel_fro(got[grp], got[1]).max():.3e}")
    assert np.all(e <= TOL), e
    assert np.all(em <= 3e-7), em
    assert np.all(rel_fro(got[grp], got[1]) <= 3e-7)
