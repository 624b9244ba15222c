"""GPU parity of the imaginary-axis correlation self-energy (Eq.(sigci),
sigc_accumulate, FP64 and BF16x3 paths) against the CPU oracle: the
integration weights alone, ragged multi-tile sizes, several problems and
blocks, workspace grouping, both FP64 kernel variants, accumulate mode,
degenerate cases, and the full-size workload on sampled entries; the BF16x3
path also against the numpy split model."""
import sys

import numpy as np
import pytest
import torch

from oracle.sigc_oracle import ag_weights, sigc_entries, sigc_ref
from gpu_common import need_gpu, rel_fro
from splitmodel import sigc_model
from paper_2506_03477_amd import Context, SigcBlock, SigcProblem
from synth import workload
from synth.gpu import device_sigc_workload, wc_block_device

pytestmark = pytest.mark.gpu
TOL = 1e-12


@pytest.fixture(scope="module")
def ctx():
    need_gpu()
    c = Context(0)
    yield c
    c.close()


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rand_block(rng, nall, nmu, nqp, nom):
    z = (rng.standard_normal((nall, nmu, nqp)) + 1j * rng.standard_normal((nall, nmu, nqp)))
    z *= np.exp(-np.arange(nmu) / 64.0)[None, :, None]
    a = rng.standard_normal((nom, nmu, nmu)) + 1j * rng.standard_normal((nom, nmu, nmu))
    wc = -(a @ np.conj(np.transpose(a, (0, 2, 1)))) / nmu
    wc *= (1.0 / (1.0 + np.arange(nom)))[:, None, None]
    return z, wc


def _run(ctx, problems, accumulate=False, precision="fp64"):
    """problems: list of (blocks [(z, wc, eps_mid, wk)], eps_qp, mesh) in numpy;
    returns the GPU outputs as numpy."""
    dev = []
    for blocks, eps_qp, mesh in problems:
        bl = [SigcBlock(torch.from_numpy(z).cuda(), torch.from_numpy(wc).cuda(), em, wk)
              for z, wc, em, wk in blocks]
        out = torch.zeros((len(eps_qp), len(eps_qp)), dtype=torch.complex128, device="cuda")
        dev.append(SigcProblem(bl, np.asarray(eps_qp), np.asarray(mesh), out))
    ctx.sigc_accumulate(dev, accumulate=accumulate, precision=precision)
    torch.cuda.synchronize()
    return dev, [p.sigc.cpu().numpy() for p in dev]


def test_weights_match_oracle(ctx):
    """One intermediate state, one product-basis function and W_i = e_j on
    the mesh: I[n][n] / (-w_k |z_n|^2) is the weight w_j(eps_n - e'), here
    for energy differences from 1e-12 to 1e3 Ha of both signs and exactly 0,
    on a mesh with and without the w = 0 node."""
    rng = np.random.default_rng(3)
    for mesh in ([0.0, 0.013, 0.072, 0.19, 0.40, 0.74, 1.35, 2.53, 5.24, 13.8, 75.6],
                 [0.05, 0.3, 1.1, 4.0], [0.0], [0.7]):
        mesh = np.array(mesh)
        mags = 10.0 ** np.linspace(-12, 3, 40)
        d = np.concatenate([mags, -mags, [0.0]])
        nqp = len(d)
        e1 = 0.25
        eps_qp = e1 + d
        d_exact = eps_qp - e1
        z = np.zeros((1, 1, nqp), complex)
        z[0, 0, :] = 1.0
        got = []
        for j in range(len(mesh)):
            wc = np.zeros((len(mesh), 1, 1), complex)
            wc[j, 0, 0] = 1.0
            _, (out,) = _run(ctx, [([(z, wc, np.array([e1]), 0.5)], eps_qp, mesh)])
            got.append(-np.real(np.diag(out)) / 0.5)
        got = np.array(got).T                                   # [n][j]
        ref = np.array([ag_weights(float(x), mesh) for x in d_exact])
        err = np.abs(got - ref) / np.maximum(np.abs(ref).max(axis=1, keepdims=True), 1e-300)
        _say(f"mesh {len(mesh)} nodes: max weight error {err.max():.2e}")
        assert err.max() < 1e-13, (mesh, np.unravel_index(err.argmax(), err.shape))
        assert np.all(got[d_exact == 0] == 0)


CASES = [
    # (nqp, [(nall, nmu)], nomega, mesh start) -- several tiles and ragged tails
    (150, [(5, 300), (3, 130)], 4, 0.0),
    (37, [(9, 200)], 3, 0.2),
    (1, [(4, 129)], 2, 0.0),
    (260, [(2, 64), (1, 1)], 1, 0.0),
    (129, [(1, 257)], 5, 0.05),
]


@pytest.mark.parametrize("case", CASES)
def test_parity_random(ctx, case):
    nqp, shapes, nom, w0 = case
    _say(f"sigc parity nqp={nqp} blocks={shapes} nomega={nom}")
    rng = np.random.default_rng(nqp * 7 + nom)
    mesh = np.cumsum(np.concatenate([[w0], rng.uniform(0.1, 1.5, nom - 1)]))
    eps_qp = np.sort(rng.uniform(-0.8, 2.0, nqp))
    blocks = []
    for nall, nmu in shapes:
        z, wc = _rand_block(rng, nall, nmu, nqp, nom)
        blocks.append((z, wc, np.sort(rng.uniform(-0.8, 3.0, nall)), float(rng.uniform(0.1, 1.0))))
    ref = sigc_ref(blocks, eps_qp, mesh)
    for variant in (0, 1):
        ctx.sigc_set_variant(variant)
        _, (out,) = _run(ctx, [(blocks, eps_qp, mesh)])
        e = rel_fro(out, ref)
        _say(f"  variant {variant}: rel Frobenius error {e:.2e}")
        assert e < TOL
        assert np.max(np.abs(out - ref)) <= TOL * np.max(np.abs(ref))
    ctx.sigc_set_variant(1)


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_several_problems_grouping_and_accumulate(ctx, precision):
    """Two problems (different nqp and meshes) in one call; one block per
    workspace group gives the same result (BF16x3: to its rounding, the
    second contraction's segments follow the grouping); accumulate adds; an
    empty problem and an empty block are handled."""
    tol = TOL if precision == "fp64" else BF16_TOL
    rng = np.random.default_rng(17)
    probs = []
    for nqp, shapes, nom in ((70, [(3, 150), (2, 90), (4, 150)], 3), (131, [(2, 140)], 2)):
        mesh = np.cumsum(rng.uniform(0.05, 1.0, nom)) - 0.05
        eps_qp = rng.uniform(-1, 1, nqp)
        blocks = []
        for nall, nmu in shapes:
            z, wc = _rand_block(rng, nall, nmu, nqp, nom)
            blocks.append((z, wc, rng.uniform(-1, 2, nall), 0.25))
        probs.append((blocks, eps_qp, mesh))
    refs = [sigc_ref(b, e, m) for b, e, m in probs]
    _, outs = _run(ctx, probs, precision=precision)
    for o, r in zip(outs, refs):
        assert rel_fro(o, r) < tol
    ctx.sigc_set_workspace_cap(1)
    try:
        dev, outs2 = _run(ctx, probs, precision=precision)
    finally:
        ctx.sigc_set_workspace_cap(0)
    for o, o2 in zip(outs, outs2):
        assert rel_fro(o2, o) < (1e-14 if precision == "fp64" else 2e-6)
    ctx.sigc_accumulate(dev, accumulate=True, precision=precision)
    torch.cuda.synchronize()
    # the default grouping again (deterministic: bit for bit outs), added
    for p, o, o2 in zip(dev, outs, outs2):
        assert rel_fro(p.sigc.cpu().numpy(), o2 + o) < 1e-15
    # a problem without blocks, and a block without intermediate states
    empty_z = torch.zeros((0, 5, 4), dtype=torch.complex128, device="cuda")
    wc = torch.zeros((2, 5, 5), dtype=torch.complex128, device="cuda")
    out_a = torch.full((4, 4), 3.0 + 1j, dtype=torch.complex128, device="cuda")
    out_b = torch.full((4, 4), 3.0 + 1j, dtype=torch.complex128, device="cuda")
    pa = SigcProblem([], np.zeros(4), np.array([0.0, 1.0]), out_a)
    pb = SigcProblem([SigcBlock(empty_z, wc, np.zeros(0), 1.0)], np.zeros(4), np.array([0.0, 1.0]), out_b)
    ctx.sigc_accumulate([pa, pb], precision=precision)
    torch.cuda.synchronize()
    assert torch.all(out_a == 0) and torch.all(out_b == 0)
    out_a.fill_(3.0 + 1j)
    ctx.sigc_accumulate([pa], accumulate=True)
    torch.cuda.synchronize()
    assert torch.all(out_a == 3.0 + 1j)


def test_degenerate_states_hermitian(ctx):
    """Equal quasiparticle energies: I^c is Hermitian; with every
    intermediate state below them and W <= 0 it is positive semidefinite."""
    rng = np.random.default_rng(23)
    nqp, nom = 40, 3
    mesh = np.array([0.0, 0.5, 2.0])
    z, wc = _rand_block(rng, 6, 70, nqp, nom)
    blocks = [(z, wc, rng.uniform(-1.0, 0.2, 6), 0.5)]
    eps_qp = np.full(nqp, 0.3)
    _, (out,) = _run(ctx, [(blocks, eps_qp, mesh)])
    assert rel_fro(out, sigc_ref(blocks, eps_qp, mesh)) < TOL
    assert np.max(np.abs(out - out.conj().T)) < 1e-12 * np.max(np.abs(out))
    ev = np.linalg.eigvalsh((out + out.conj().T) / 2)
    assert ev.min() > -1e-12 * ev.max()


def test_synthetic_generator_matches_cpu(ctx):
    wl = workload(6).replace(npb=9, nocc=3, nunocc=150)
    blk = wl.blocks()[2]
    w_dev = wc_block_device(wl, blk).cpu().numpy()
    assert np.array_equal(w_dev, wl.wc_block(blk))


def test_reduced_workload(ctx):
    """Workload 6 at reduced sizes (inputs from the device generators, the
    oracle from the CPU generators)."""
    wl = workload(6).replace(npb=150, nocc=24, nunocc=260, nk=3, nval=8)
    _say(f"reduced workload {wl.npb} x {wl.nocc} x {wl.nunocc}, nk {wl.nk}")
    blks, eps_qp = device_sigc_workload(wl)
    out = torch.empty((wl.npb, wl.npb), dtype=torch.complex128, device="cuda")
    prob = SigcProblem([SigcBlock(z, wc, em, wk) for z, wc, em, wk, _ in blks], eps_qp,
                       wl.omega_array(), out)
    ctx.sigc_accumulate([prob])
    torch.cuda.synchronize()
    ref = sigc_ref(((wl.z_block(b).astype(np.complex128), wl.wc_block(b), wl.eps_mid(b), b.wk)
                    for b in wl.blocks()), wl.eps_qp(), wl.omega)
    e = rel_fro(out.cpu().numpy(), ref)
    _say(f"  rel Frobenius error {e:.2e}")
    assert e < TOL


def test_full_size_sampled(ctx):
    """Workload 6 at full size (nqp 206, nall 361, 1356 product-basis
    functions, 16 k-points, 11 frequencies) in the launch configuration the
    benchmark times; entries on and off the diagonal, occupied and
    unoccupied rows, checked against the oracle evaluated entry by entry."""
    wl = workload(6)
    _say(f"full-size {wl.name}: generating inputs on the device")
    blks, eps_qp = device_sigc_workload(wl)
    out = torch.empty((wl.npb, wl.npb), dtype=torch.complex128, device="cuda")
    prob = SigcProblem([SigcBlock(z, wc, em, wk) for z, wc, em, wk, _ in blks], eps_qp,
                       wl.omega_array(), out)
    ctx.sigc_accumulate([prob])
    torch.cuda.synchronize()
    got_full = out.cpu().numpy()
    del blks, prob
    torch.cuda.empty_cache()
    entries = [(0, 0), (91, 92), (92, 91), (205, 205), (17, 150), (150, 17), (100, 3)]
    cols = sorted({c for e in entries for c in e})

    def blocks():
        for b in wl.blocks():
            pairs = np.arange(b.npairs)
            zc = wl.z_elements(b, pairs, np.array(cols)).reshape(b.nocc, b.nunocc, len(cols))
            yield zc, cols, wl.wc_block(b), wl.eps_mid(b), b.wk
    _say("  oracle entries")
    ref = sigc_entries(blocks(), wl.eps_qp(), wl.omega, entries)
    got = np.array([got_full[n, m] for n, m in entries])
    e = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    _say(f"  sampled rel error {e:.2e}; |I| max {np.abs(got_full).max():.3e}")
    assert e < TOL
    assert np.all(np.isfinite(got_full))


# BF16x3 contractions.  Every operand keeps 16 significant bits (hi + lo of
# its FP32 value), so a product carries a random relative error of about
# 4e-6; the entries of Z_w^H W^c and of I^c are sums of terms of both signs,
# which keep that relative error instead of averaging it down (unlike the
# positive diagonal of chi0), and the two contractions' errors add in
# quadrature (about 5.7e-6 at most).  Bound against the oracle: 8e-6 relative
# Frobenius.  Against the split model (the kernels' roundings, exact
# products, FP64 sums) only the FP32 runs of at most 4096 rows differ:
# relative u sqrt(run) ~ 4e-6 at most, bound 4e-6.
BF16_TOL = 8e-6
BF16_MODEL_TOL = 4e-6


@pytest.mark.parametrize("case", CASES + [(96, [(4, 520)], 3, 0.0)])
def test_bf16x3_parity(ctx, case):
    nqp, shapes, nom, w0 = case
    _say(f"sigc bf16x3 nqp={nqp} blocks={shapes} nomega={nom}")
    rng = np.random.default_rng(nqp * 11 + nom)
    mesh = np.cumsum(np.concatenate([[w0], rng.uniform(0.1, 1.5, nom - 1)]))
    eps_qp = np.sort(rng.uniform(-0.8, 2.0, nqp))
    blocks = []
    for nall, nmu in shapes:
        z, wc = _rand_block(rng, nall, nmu, nqp, nom)
        blocks.append((z, wc, np.sort(rng.uniform(-0.8, 3.0, nall)), float(rng.uniform(0.1, 1.0))))
    ref = sigc_ref(blocks, eps_qp, mesh)
    model = sigc_model(blocks, eps_qp, mesh)
    _, (out,) = _run(ctx, [(blocks, eps_qp, mesh)], precision="bf16x3")
    e, em = rel_fro(out, ref), rel_fro(out, model)
    _say(f"  vs oracle {e:.2e}, vs split model {em:.2e}, model vs oracle {rel_fro(model, ref):.2e}")
    assert e < BF16_TOL and em < BF16_MODEL_TOL


def test_bf16x3_reduced_workload(ctx):
    wl = workload(6).replace(npb=150, nocc=24, nunocc=260, nk=3, nval=8)
    blks, eps_qp = device_sigc_workload(wl)
    out = torch.empty((wl.npb, wl.npb), dtype=torch.complex128, device="cuda")
    prob = SigcProblem([SigcBlock(z, wc, em, wk) for z, wc, em, wk, _ in blks], eps_qp,
                       wl.omega_array(), out)
    ctx.sigc_accumulate([prob], precision="bf16x3")
    torch.cuda.synchronize()
    cpu = [(wl.z_block(b).astype(np.complex128), wl.wc_block(b), wl.eps_mid(b), b.wk) for b in wl.blocks()]
    ref = sigc_ref(cpu, wl.eps_qp(), wl.omega)
    model = sigc_model(cpu, wl.eps_qp(), wl.omega)
    got = out.cpu().numpy()
    e, em = rel_fro(got, ref), rel_fro(got, model)
    _say(f"reduced workload bf16x3: vs oracle {e:.2e}, vs model {em:.2e}")
    assert e < BF16_TOL and em < BF16_MODEL_TOL


@pytest.mark.parametrize("precision", ["fp64", "bf16x3"])
def test_zero_and_tiny_energy_differences(ctx, precision):
    """Energy differences exactly 0 (all weights 0) and 1e-300 (weights of
    very different sizes) next to ordinary ones: the BF16x3 path multiplies
    Z by the weights before rounding it to FP32, where products with a
    weight of 1e-300 become 0 (terms far below the tolerance), and sums all
    mesh points in one run."""
    rng = np.random.default_rng(41)
    nqp, nom = 70, 5
    mesh = np.array([0.0, 0.2, 0.7, 2.0, 9.0])
    z, wc = _rand_block(rng, 4, 180, nqp, nom)
    eps_mid = np.array([0.0, 0.4, -0.3, 1.1])
    eps_qp = np.sort(rng.uniform(-0.8, 2.0, nqp))
    eps_qp[3] = 0.4                      # dE = 0 against n' = 1
    eps_qp[5] = 1e-300                   # dE = 1e-300 against n' = 0
    eps_qp[6] = -1e-300
    blocks = [(z, wc, eps_mid, 0.5)]
    ref = sigc_ref(blocks, eps_qp, mesh)
    _, (out,) = _run(ctx, [(blocks, eps_qp, mesh)], precision=precision)
    e = rel_fro(out, ref)
    tol = TOL if precision == "fp64" else BF16_TOL
    _say(f"zero / tiny dE, {precision}: {e:.2e}")
    assert e < tol
    if precision == "bf16x3":
        assert rel_fro(out, sigc_model(blocks, eps_qp, mesh)) < BF16_MODEL_TOL
