"""Full-size parity at the workload sizes the benchmark times (npb = 2048,
16 k-blocks of 200 x 1200 pairs, 12 frequencies), in the same launch
configuration: sampled chi0 entries computed one by one by the oracle, plus
properties that hold at any size (exact Hermiticity, eps built exactly from
chi0, inverse residual)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from gpu_common import assert_hermitian_exact, device_problem, need_gpu
from paper_2506_03477_amd import Context
from synth import workload

pytestmark = pytest.mark.gpu

# entries: diagonal, tile corners and ragged boundaries, far off-diagonal
ENTRIES = [(0, 0), (1, 0), (127, 127), (128, 127), (128, 128), (255, 1), (1000, 999),
           (1024, 0), (2047, 2047), (2047, 0), (1500, 700), (64, 63), (513, 511), (2046, 129)]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _oracle_entries(wl):
    cols = sorted({i for e in ENTRIES for i in e})
    col_index = {c: k for k, c in enumerate(cols)}

    def gen():
        for blk in wl.blocks(0):
            eo, eu = wl.energies(blk)
            yield wl.z_elements(blk, np.arange(blk.npairs), np.array(cols)), eo, eu, blk.wk
    return oracle.chi0_entries(gen(), ENTRIES, col_index, wl.omega, wl.delta_min)


def _normalized_errors(chi, ref_entries, ref_diag):
    errs = []
    for k, (i, j) in enumerate(ENTRIES):
        scale = np.sqrt(np.abs(ref_diag[:, i]) * np.abs(ref_diag[:, j]))
        errs.append(np.abs(chi[:, i, j] - ref_entries[:, k]) / scale)
    return np.array(errs)


@pytest.fixture(scope="module")
def ref():
    need_gpu()
    wl = workload(2)
    _say("oracle: sampled entries of the npb=2048 workload")
    return wl, _oracle_entries(wl)


@pytest.mark.parametrize("path,tol", [("bf16x3", 1e-6), ("fp64", 1e-12)])
def test_fullsize_sampled_entries(ref, path, tol):
    wl, ent = ref
    ztype = "c128" if path == "fp64" else "c64"
    _say(f"full size {wl.name} {path}")
    ctx = Context(0)
    prob, vsqrt, _ = device_problem(wl, ztype=ztype)
    ctx.chi0_accumulate([prob], precision=path, delta_min=wl.delta_min)
    ctx.sync()
    chi = prob.chi0
    assert_hermitian_exact(chi)
    idx_i = torch.tensor([i for i, _ in ENTRIES], device=chi.device)
    idx_j = torch.tensor([j for _, j in ENTRIES], device=chi.device)
    got = chi[:, idx_i, idx_j].cpu().numpy()                   # [nomega, nentries]
    diag = torch.diagonal(chi, dim1=1, dim2=2).cpu().numpy()
    ref_diag = {i: ent[:, k] for k, (i, j) in enumerate(ENTRIES) if i == j}
    errs = []
    for k, (i, j) in enumerate(ENTRIES):
        di = ref_diag.get(i, diag[:, i])
        dj = ref_diag.get(j, diag[:, j])
        errs.append(np.abs(got[:, k] - ent[:, k]) / np.sqrt(np.abs(di) * np.abs(dj)))
    errs = np.array(errs)
    _say(f"  max normalized entry error {errs.max():.3e} (tol {tol})")
    assert errs.max() <= tol, errs
    if path == "bf16x3":
        # dielectric step at full size: eps exactly from chi0, inverse residual
        inv = torch.empty_like(chi)
        eps = torch.empty_like(chi)
        ctx.dielectric_invert(vsqrt, chi, inv, eps=eps)
        ctx.sync()
        for iw in (0, wl.nomega // 2, wl.nomega - 1):
            e_ref = oracle.dielectric(chi[iw:iw + 1].cpu().numpy(), wl.vsqrt())[0]
            e_gpu = eps[iw].cpu().numpy()
            assert np.array_equal(e_gpu, e_ref)
            x = inv[iw].cpu().numpy()
            res = np.linalg.norm(e_gpu @ x - np.eye(wl.npb)) / np.sqrt(wl.npb)
            kappa_bound = np.linalg.norm(e_gpu)             # lambda_min(eps) >= 1, ||.||_2 <= ||.||_F
            _say(f"  iw={iw} residual {res:.3e} kappa<={kappa_bound:.3e}")
            assert res <= 64 * wl.npb * kappa_bound * np.finfo(float).eps
            asym = np.linalg.norm(x - x.conj().T) / np.linalg.norm(x)
            assert asym <= 64 * wl.npb * kappa_bound * np.finfo(float).eps, asym
    del prob
    ctx.close()
    torch.cuda.empty_cache()
