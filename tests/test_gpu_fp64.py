"""GPU parity of the FP64 path and of the dielectric step against the CPU
oracle (element by element, relative Frobenius error per frequency)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_common import (assert_hermitian_exact, device_problem, need_gpu, oracle_chi0,
                        rel_fro)
from paper_2506_03477_amd import Block, Chi0Error, Context, Problem, CHI0_ENOTHPD, CHI0_ESINGULAR
from synth import workload
from synth.gpu import z_block_device

pytestmark = pytest.mark.gpu
TOL_FP64 = 1e-12


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    c = Context(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_synth_gpu_matches_cpu():
    need_gpu()
    for wl in (workload(0), workload(2, npb=96, nocc=5, nunocc=33)):
        blk = wl.blocks()[1]
        _say(f"synth {wl.name} {wl.ztype}")
        zg = z_block_device(wl, blk).cpu().numpy()
        zc = wl.z_block(blk)
        assert zg.dtype == zc.dtype
        assert np.array_equal(zg.view(np.uint8), zc.view(np.uint8))


def _run(ctx, wl, prec="fp64", ztype=None, **kw):
    prob, vsqrt, blks = device_problem(wl, ztype=ztype)
    ctx.chi0_accumulate([prob], precision=prec, delta_min=wl.delta_min, **kw)
    ctx.sync()
    return prob, vsqrt


@pytest.mark.parametrize("cfg,over", [
    (0, {}),                                                     # npb 64 workload, full size
    (1, dict(npb=200, nk=3, nocc=7, nunocc=45)),                 # ragged npb, several tiles
    (3, dict(nq=1, npb=130, nk=5, ztype="c128")),                # uneven blocks
    (4, dict(npb=96, nk=3, ztype="c128")),                       # spins, intraband cut
])
def test_fp64_parity(ctx, cfg, over):
    wl = workload(cfg, **over)
    _say(f"fp64 parity {wl.name} {over}")
    prob, _ = _run(ctx, wl)
    got = prob.chi0.cpu().numpy()
    ref = oracle_chi0(wl)
    err = rel_fro(got, ref)
    _say(f"  rel err per omega: {err}")
    assert np.all(err <= TOL_FP64), err
    assert_hermitian_exact(prob.chi0)


def test_fp64_tile_configs_agree(ctx):
    wl = workload(1, npb=100, nk=2, nocc=6, nunocc=40)
    ref = oracle_chi0(wl)
    for t in range(ctx.tile_count("fp64")):
        _say(f"fp64 tile {t} {ctx.tile_info('fp64', t)}")
        ctx.set_tile("fp64", t)
        prob, _ = _run(ctx, wl)
        assert np.all(rel_fro(prob.chi0.cpu().numpy(), ref) <= TOL_FP64)
    ctx.set_tile("fp64", -1)


def test_fp64_accumulate_deterministic_and_graph(ctx):
    wl = workload(1, npb=150, nk=4, nocc=6, nunocc=30)
    _say("fp64 accumulate/determinism/graph")
    prob, _, blks = device_problem(wl)
    ctx.chi0_accumulate([prob])
    first = prob.chi0.clone()
    ctx.chi0_accumulate([prob])
    torch.cuda.synchronize()
    assert torch.equal(first, prob.chi0)                      # bitwise deterministic
    # two accumulate calls over halves of the blocks == one call (to rounding)
    half = len(prob.blocks) // 2
    p1 = Problem(prob.blocks[:half], prob.omega, torch.zeros_like(prob.chi0))
    ctx.chi0_accumulate([p1])
    p2 = Problem(prob.blocks[half:], prob.omega, p1.chi0)
    ctx.chi0_accumulate([p2], accumulate=True)
    ctx.sync()
    assert np.all(rel_fro(p2.chi0.cpu().numpy(), first.cpu().numpy()) <= 1e-14)
    assert_hermitian_exact(p2.chi0)
    # streaming one k-block per call (accumulate mode) == one call (to rounding)
    ps = Problem(prob.blocks[:1], prob.omega, torch.zeros_like(prob.chi0))
    ctx.chi0_accumulate([ps])
    for b in prob.blocks[1:]:
        ctx.chi0_accumulate([Problem([b], prob.omega, ps.chi0)], accumulate=True)
    ctx.sync()
    assert np.all(rel_fro(ps.chi0.cpu().numpy(), first.cpu().numpy()) <= 1e-14)
    # graph replays (with eager work in between) reproduce the direct result
    for rep in range(3):
        prob.chi0.fill_(7.0)
        ctx.chi0_accumulate([prob], graph=True)
        torch.cuda.synchronize()
        junk = torch.randn(1000, device="cuda").sum()
        assert torch.equal(prob.chi0, first), rep
    ctx.sync()


def test_fp64_batched_problems(ctx):
    _say("fp64 batched problems")
    wls = [workload(3, nq=3, npb=npb, nk=3, ztype="c128", omega=om)
           for npb, om in ((64, (0.1, 1.0)), (130, (0.05,)), (97, (0.2, 0.7, 3.0)))]
    probs, refs = [], []
    for q, wl in enumerate(wls):
        prob, _, _ = device_problem(wl, q=q)
        probs.append(prob)
        refs.append(oracle_chi0(wl, q=q))
    ctx.chi0_accumulate(probs)
    ctx.sync()
    for prob, ref in zip(probs, refs):
        assert np.all(rel_fro(prob.chi0.cpu().numpy(), ref) <= TOL_FP64)
        assert_hermitian_exact(prob.chi0)


def test_fp64_empty_and_tiny(ctx):
    _say("fp64 empty/tiny")
    dev = "cuda"
    om = torch.tensor([0.0, 1.0], dtype=torch.float64, device=dev)
    # npb = 1, one pair, omega = 0: chi0 = -2 wk |z|^2 / D
    z = torch.tensor([[[1.0 + 2.0j]]], dtype=torch.complex128, device=dev)
    eo = torch.tensor([-0.25], dtype=torch.float64, device=dev)
    eu = torch.tensor([0.25], dtype=torch.float64, device=dev)
    chi = torch.empty((2, 1, 1), dtype=torch.complex128, device=dev)
    empty = Block(None, torch.empty(0, dtype=torch.float64, device=dev),
                  torch.empty(0, dtype=torch.float64, device=dev), 1.0)
    ctx.chi0_accumulate([Problem([empty, Block(z, eo, eu, 0.5), empty], om, chi)])
    ctx.sync()
    got = chi.cpu().numpy()[:, 0, 0]
    assert got[0] == -10.0                       # f(D, 0) = -2 wk / D = -2, |z|^2 = 5
    assert abs(got[1] - (-2.0)) <= 1e-15            # f(D, 1) = -0.4
    # a problem with no pairs writes zeros
    chi.fill_(3.0)
    ctx.chi0_accumulate([Problem([empty], om, chi)])
    ctx.sync()
    assert torch.all(chi == 0)


def _dielectric(ctx, wl):
    prob, vsqrt, _ = device_problem(wl)
    ctx.chi0_accumulate([prob], delta_min=wl.delta_min)
    eps = torch.empty_like(prob.chi0)
    inv = torch.empty_like(prob.chi0)
    wc = torch.empty_like(prob.chi0)
    ctx.dielectric_invert(vsqrt, prob.chi0, inv, eps=eps, wc=wc)
    ctx.sync()
    return prob.chi0.cpu().numpy(), eps.cpu().numpy(), inv.cpu().numpy(), wc.cpu().numpy()


@pytest.mark.parametrize("cfg,over", [(0, {}), (1, dict(npb=150, nk=2, nocc=8, nunocc=40))])
def test_dielectric_parity(ctx, cfg, over):
    wl = workload(cfg, **over)
    _say(f"dielectric {wl.name}")
    chi, eps, inv, wc = _dielectric(ctx, wl)
    s = wl.vsqrt()
    eps_ref = oracle.dielectric(chi, s)            # same chi0: exact same eps expected
    assert np.array_equal(eps, eps_ref)
    chi_ref = oracle_chi0(wl)
    eps_o = oracle.dielectric(chi_ref, s)
    inv_ref = oracle.inverse(eps_o, "lapack")
    u = np.finfo(float).eps / 2
    for iw in range(wl.nomega):
        kappa = np.linalg.cond(eps_o[iw])
        tol = max(TOL_FP64, 64 * kappa * u)
        e = rel_fro(inv[iw], inv_ref[iw])
        res = np.linalg.norm(eps[iw] @ inv[iw] - np.eye(wl.npb)) / np.sqrt(wl.npb)
        _say(f"  iw={iw} kappa={kappa:.3g} inv rel={e:.3g} tol={tol:.3g} residual={res:.3g}")
        assert e <= tol
        assert res <= 64 * wl.npb * kappa * u
    wc_ref = oracle.screened_wc(inv, s)
    assert np.array_equal(wc, wc_ref)               # W^c from the same eps^-1: bitwise


def test_dielectric_singular(ctx):
    _say("dielectric singular")
    n = 8
    s = torch.full((n,), 0.5, dtype=torch.float64, device="cuda")
    chi = torch.zeros((1, n, n), dtype=torch.complex128, device="cuda")
    chi[0].diagonal().fill_(4.0)                    # eps = 1 - 0.25 * 4 = 0
    inv = torch.empty_like(chi)
    ctx.dielectric_invert(s, chi, inv)
    with pytest.raises(Chi0Error) as ei:
        ctx.sync()
    assert ei.value.code == CHI0_ESINGULAR
    ctx.sync()                                      # status is cleared once reported


def _nsd_chi0(n, nomega, seed):
    """A negative semidefinite Hermitian chi0 (-A^H diag(c) A, c > 0) of
    rank min(n, 3n/2) per frequency, and the Coulomb square roots 1/(1+I)."""
    rng = np.random.default_rng(seed)
    k = max(1, 3 * n // 2)
    out = np.empty((nomega, n, n), np.complex128)
    for iw in range(nomega):
        a = rng.standard_normal((k, n)) + 1j * rng.standard_normal((k, n))
        c = rng.uniform(0.1, 2.0, k) / (1.0 + iw)
        out[iw] = -(a.conj().T * c) @ a
    return out, 1.0 / (1.0 + np.arange(n, dtype=np.float64))


def _check_hpd_inverse(eps, inv, eps_o, tag):
    u = np.finfo(float).eps / 2
    inv_ref = oracle.inverse(eps_o, "cholesky")
    n = eps.shape[-1]
    for iw in range(eps.shape[0]):
        kappa = np.linalg.cond(eps_o[iw])
        tol = max(TOL_FP64, 64 * kappa * u)
        e = rel_fro(inv[iw], inv_ref[iw])
        res = np.linalg.norm(eps[iw] @ inv[iw] - np.eye(n)) / np.sqrt(n)
        _say(f"  {tag} iw={iw} kappa={kappa:.3g} inv rel={e:.3g} residual={res:.3g}")
        assert e <= tol
        assert res <= 64 * n * kappa * u
        assert np.array_equal(inv[iw], inv[iw].conj().T)     # mirrored: exactly Hermitian
        assert np.all(np.diag(inv[iw]).imag == 0)


@pytest.mark.parametrize("n", [1, 7, 8, 9, 31, 32, 33, 40, 100, 130])
def test_dielectric_gj_sizes_pivoting(ctx, n):
    """Pivoted Gauss-Jordan inverse of a general (non-Hermitian) eps whose
    off-diagonal entries are as large as its diagonal, so rows are
    interchanged, at sizes that end a panel (32 columns) or a sub-panel (8
    columns) early, exactly, or one column late; against the oracle's
    textbook Gauss-Jordan."""
    _say(f"dielectric gj n={n}")
    rng = np.random.default_rng(1000 + n)
    chi_h = (rng.standard_normal((2, n, n)) + 1j * rng.standard_normal((2, n, n))) * (2.0 / np.sqrt(n))
    s_h = np.ones(n)
    chi = torch.from_numpy(chi_h).cuda()
    s = torch.from_numpy(s_h).cuda()
    eps = torch.empty_like(chi)
    inv = torch.empty_like(chi)
    ctx.dielectric_invert(s, chi, inv, eps=eps, method="gj")
    ctx.sync()
    eps_o = oracle.dielectric(chi_h, s_h)
    assert np.array_equal(eps.cpu().numpy(), eps_o)
    inv_ref = oracle.inverse(eps_o, "gauss_jordan")
    got = inv.cpu().numpy()
    u = np.finfo(float).eps / 2
    for iw in range(2):
        kappa = np.linalg.cond(eps_o[iw])
        e = rel_fro(got[iw], inv_ref[iw])
        res = np.linalg.norm(eps_o[iw] @ got[iw] - np.eye(n)) / np.sqrt(n)
        _say(f"  iw={iw} kappa={kappa:.3g} inv rel={e:.3g} residual={res:.3g}")
        assert e <= max(TOL_FP64, 64 * kappa * u)
        assert res <= 64 * n * kappa * u


@pytest.mark.parametrize("n", [1, 31, 32, 33, 63, 64, 65, 100, 129, 130, 200])
def test_dielectric_hpd_sizes(ctx, n):
    """Hermitian positive definite inverse (symmetric sweeps) at block-
    ragged sizes, against the oracle's Cholesky inverse."""
    _say(f"dielectric hpd n={n}")
    chi_h, s_h = _nsd_chi0(n, 3, seed=n)
    chi = torch.from_numpy(chi_h).cuda()
    s = torch.from_numpy(s_h).cuda()
    eps = torch.empty_like(chi)
    inv = torch.empty_like(chi)
    wc = torch.empty_like(chi)
    ctx.dielectric_invert(s, chi, inv, eps=eps, wc=wc, method="hpd")
    ctx.sync()
    eps_o = oracle.dielectric(chi_h, s_h)
    assert np.array_equal(eps.cpu().numpy(), eps_o)
    _check_hpd_inverse(eps.cpu().numpy(), inv.cpu().numpy(), eps_o, f"n={n}")
    assert np.array_equal(wc.cpu().numpy(), oracle.screened_wc(inv.cpu().numpy(), s_h))


@pytest.mark.parametrize("cfg,over", [(0, {}), (1, dict(npb=150, nk=2, nocc=8, nunocc=40))])
def test_dielectric_hpd_parity(ctx, cfg, over):
    wl = workload(cfg, **over)
    _say(f"dielectric hpd {wl.name}")
    prob, vsqrt, _ = device_problem(wl)
    ctx.chi0_accumulate([prob], delta_min=wl.delta_min)
    eps = torch.empty_like(prob.chi0)
    inv = torch.empty_like(prob.chi0)
    inv_gj = torch.empty_like(prob.chi0)
    ctx.dielectric_invert(vsqrt, prob.chi0, inv, eps=eps, method="hpd")
    ctx.dielectric_invert(vsqrt, prob.chi0, inv_gj, method="gj")
    ctx.sync()
    s = wl.vsqrt()
    eps_o = oracle.dielectric(oracle_chi0(wl), s)
    _check_hpd_inverse(eps.cpu().numpy(), inv.cpu().numpy(), eps_o, wl.name)
    u = np.finfo(float).eps / 2
    for iw in range(wl.nomega):
        kappa = np.linalg.cond(eps_o[iw])
        assert rel_fro(inv.cpu().numpy()[iw], inv_gj.cpu().numpy()[iw]) <= max(TOL_FP64, 64 * kappa * u)


def test_dielectric_hpd_rejects_indefinite(ctx):
    """An indefinite eps is reported (CHI0_ENOTHPD); the fallback method
    returns the pivoted Gauss-Jordan inverse instead, bit for bit."""
    _say("dielectric hpd indefinite / fallback")
    n = 40
    chi_h, s_h = _nsd_chi0(n, 2, seed=7)
    chi_h[0] = -chi_h[0] * 50.0                       # eps = 1 - 50 s A^H c A s: indefinite
    chi = torch.from_numpy(chi_h).cuda()
    s = torch.from_numpy(s_h).cuda()
    inv = torch.empty_like(chi)
    ctx.dielectric_invert(s, chi, inv, method="hpd")
    with pytest.raises(Chi0Error) as ei:
        ctx.sync()
    assert ei.value.code == CHI0_ENOTHPD
    ctx.sync()                                        # cleared once reported
    inv_fb = torch.empty_like(chi)
    inv_gj = torch.empty_like(chi)
    ctx.dielectric_invert(s, chi, inv_fb, method="hpd_fallback_gj")
    ctx.dielectric_invert(s, chi, inv_gj, method="gj")
    ctx.sync()                                        # the fallback reports nothing
    assert torch.equal(inv_fb, inv_gj)
    eps_o = oracle.dielectric(chi_h, s_h)
    ref = oracle.inverse(eps_o, "lapack")
    for iw in range(2):
        assert rel_fro(inv_gj.cpu().numpy()[iw], ref[iw]) <= 1e-10
