"""Edge cases through the C ABI on the GPU, all three precisions: npb = 1 and
tile-boundary sizes, one frequency, omega = 0, every pair cut by delta_min,
empty problems next to non-empty ones."""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_common import assert_hermitian_exact, device_problem, need_gpu, oracle_chi0, rel_fro
from paper_2506_03477_amd import Block, Context, Problem
from synth import workload

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 3e-6}
ZT = {"fp64": "c128", "fp32": "c64", "bf16x3": "c64"}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    c = Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("path", ["fp64", "fp32", "bf16x3"])
@pytest.mark.parametrize("npb", [1, 31, 64, 65, 127, 128, 129, 257])
def test_tile_boundary_sizes(ctx, path, npb):
    wl = workload(0, npb=npb, nk=4, nocc=6, nunocc=50, ztype=ZT[path], omega=(0.0, 0.3))
    prob, _, _ = device_problem(wl)
    ctx.chi0_accumulate([prob], precision=path)
    ctx.sync()
    ref = oracle_chi0(wl)
    err = rel_fro(prob.chi0.cpu().numpy(), ref)
    _say(f"{path} npb={npb}: {err.max():.3e}")
    # BF16x3 floor ~4e-6 sqrt(npb / K): K = 1200 here
    tol = TOL[path] if path != "bf16x3" else max(TOL[path], 8e-6 * np.sqrt(npb / 1200))
    assert np.all(err <= tol)
    assert_hermitian_exact(prob.chi0)


@pytest.mark.parametrize("path", ["fp64", "fp32", "bf16x3"])
def test_all_pairs_cut_and_empty_problems(ctx, path):
    wl = workload(1, npb=70, nk=2, nocc=5, nunocc=20, ztype=ZT[path])
    live, _, _ = device_problem(wl)
    cut, _, _ = device_problem(wl)            # same blocks, delta_min above every D
    dev = "cuda"
    empty = Problem([], torch.tensor([1.0], dtype=torch.float64, device=dev),
                    torch.full((1, 33, 33), 5.0, dtype=torch.complex128, device=dev))
    ctx.chi0_accumulate([cut], precision=path, delta_min=100.0)
    ctx.sync()
    assert torch.all(cut.chi0 == 0)
    ctx.chi0_accumulate([empty, live], precision=path)
    ctx.sync()
    assert torch.all(empty.chi0 == 0)
    tol = {"fp64": 1e-12, "fp32": 1e-6, "bf16x3": 1e-5}[path]   # K = 200 pairs only
    assert np.all(rel_fro(live.chi0.cpu().numpy(), oracle_chi0(wl)) <= tol)


def test_mixed_problem_shapes_one_call(ctx):
    shapes = [(1, (0.5,)), (129, (0.0, 1.0, 4.0)), (40, (2.0,))]
    wls = [workload(3, nq=3, npb=npb, nk=2, omega=om, ztype="c64") for npb, om in shapes]
    probs = [device_problem(wl, q=q)[0] for q, wl in enumerate(wls)]
    ctx.chi0_accumulate(probs, precision="fp32")
    ctx.sync()
    for q, (wl, prob) in enumerate(zip(wls, probs)):
        assert np.all(rel_fro(prob.chi0.cpu().numpy(), oracle_chi0(wl, q=q)) <= 1e-6)
