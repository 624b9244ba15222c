"""Full-size parity at the sizes the benchmark times: npb = 2048, 16 k-blocks
of 200 x 1200 pairs (3.84 M pairs), 12 frequencies, complex64 Z, in the
benchmark's launch configuration (every block in one call, default tiles).

* Whole matrices: the oracle's chi0 at the smallest and the largest
  frequency (per-block FP64 products, Eq.(polfx) at i*omega, over Z copied
  back from the device in chunks and upcast exactly to complex128; the
  device generator is bit-identical to the CPU one) against the BF16x3 path
  and against the FP64 path run on the same values upcast to complex128:
  relative Frobenius error <= 1e-6 and <= 1e-12 per frequency.
* eps^-1 at both frequencies: LAPACK's inverse of the oracle's eps
  (Eq.(dielectricfunction)) against the library's inverses of the GPU chi0
  (HPD sweeps with the pivoted fall-back, the benchmark's inverse, and
  pivoted Gauss-Jordan): <= 1e-6 for BF16x3, max(1e-12, 64 kappa u) for
  FP64; the stricter ||d eps^-1|| / ||eps^-1 - 1|| is printed.
* Whole rows at every frequency: the oracle's rows of chi0 for a set of
  basis functions spanning the tile grid, against both paths.
* Both paths over whole matrices at every frequency: BF16x3 within 1e-6 of
  FP64 (the FP64 path being itself pinned above at two frequencies)."""
import numpy as np
import pytest
import torch

import oracle
from gpu_common import assert_hermitian_exact, device_problem, host_blocks, need_gpu
from paper_2506_03477_amd import Block, Context, Problem
from synth import workload

pytestmark = pytest.mark.gpu

ROWS = [0, 1, 127, 128, 255, 256, 700, 1024, 1500, 2047]
U = np.finfo(np.float64).eps / 2


def _rel(x, ref):
    return np.linalg.norm(x - ref) / np.linalg.norm(ref)


@pytest.mark.timeout(1200)
def test_fullsize_full_matrices(say):
    need_gpu()
    wl = workload(2)                                     # c64, the benchmark workload
    assert (wl.npb, wl.nk, wl.nomega) == (2048, 16, 12)
    ctx = Context(0)
    say(f"full size {wl.name}: generating complex64 Z on the device")
    prob, vsqrt, blks = device_problem(wl, ztype="c64")
    ctx.chi0_accumulate([prob], precision="bf16x3", delta_min=wl.delta_min)
    ctx.sync()
    chi_bf = prob.chi0
    assert_hermitian_exact(chi_bf)
    say("BF16x3 chi0 done; FP64 path on the same values upcast to complex128")
    z128 = [b[0].to(torch.complex128) for b in blks]
    chi_fp = torch.empty_like(chi_bf)
    p64 = Problem([Block(z, b[1], b[2], b[3]) for z, b in zip(z128, blks)], prob.omega, chi_fp)
    ctx.chi0_accumulate([p64], precision="fp64", delta_min=wl.delta_min)
    ctx.sync()
    del p64, z128
    torch.cuda.empty_cache()
    assert_hermitian_exact(chi_fp)

    # both paths over whole matrices, every frequency
    d = torch.linalg.norm((chi_bf - chi_fp).reshape(wl.nomega, -1), dim=1)
    n = torch.linalg.norm(chi_fp.reshape(wl.nomega, -1), dim=1)
    bf_vs_fp = (d / n).cpu().numpy()
    say(f"BF16x3 vs FP64 per omega: {np.array2string(bf_vs_fp, precision=2)}")
    assert np.all(bf_vs_fp <= 1e-6), bf_vs_fp

    # inverses on the GPU (all frequencies), kept at the two checked ones
    sel = [0, wl.nomega - 1]
    inv = {}
    for path, chi in (("bf16x3", chi_bf), ("fp64", chi_fp)):
        for method in ("hpd_fallback_gj", "gj"):
            out = torch.empty_like(chi)
            ctx.dielectric_invert(vsqrt, chi, out, method=method)
            ctx.sync()
            inv[path, method] = out[sel].cpu().numpy()
            del out
    got = {"bf16x3": chi_bf[sel].cpu().numpy(), "fp64": chi_fp[sel].cpu().numpy()}
    rows_got = {"bf16x3": chi_bf[:, ROWS, :].cpu().numpy(), "fp64": chi_fp[:, ROWS, :].cpu().numpy()}
    del chi_bf, chi_fp
    torch.cuda.empty_cache()

    # oracle: whole rows at every frequency, then whole matrices at two
    omega = list(wl.omega)
    say(f"oracle rows {ROWS} at all {wl.nomega} frequencies")
    ref_rows = oracle.chi0_rows(host_blocks(blks, 50), ROWS, wl.npb, omega, wl.delta_min)
    for path, tol in (("bf16x3", 1e-6), ("fp64", 1e-12)):
        e = np.array([_rel(rows_got[path][iw], ref_rows[iw]) for iw in range(wl.nomega)])
        say(f"{path} rows vs oracle per omega: {np.array2string(e, precision=2)}")
        assert np.all(e <= tol), (path, e)
    say(f"oracle full chi0 at omega = {omega[0]:.6g} and {omega[-1]:.6g} (about 4 min on 16 threads)")
    ref = oracle.chi0_ref(host_blocks(blks, 25, say, "oracle"), wl.npb, [omega[i] for i in sel],
                          wl.delta_min)
    del blks, prob
    torch.cuda.empty_cache()
    for path, tol in (("bf16x3", 1e-6), ("fp64", 1e-12)):
        e = oracle.rel_fro(got[path], ref)
        say(f"{path} chi0 vs oracle (whole matrices): {e}")
        assert np.all(e <= tol), (path, e)

    s = wl.vsqrt()
    eps_ref = oracle.dielectric(ref, s)
    inv_ref = oracle.inverse(eps_ref, "lapack")
    for k, iw in enumerate(sel):
        ev = np.linalg.eigvalsh(eps_ref[k])
        kappa = ev[-1] / ev[0]
        eye = np.eye(wl.npb)
        for (path, method), x in inv.items():
            e = _rel(x[k], inv_ref[k])
            strict = np.linalg.norm(x[k] - inv_ref[k]) / np.linalg.norm(inv_ref[k] - eye)
            tol = 1e-6 if path == "bf16x3" else max(1e-12, 64 * kappa * U)
            say(f"{path} eps^-1 ({method}) omega index {iw}: rel {e:.3e}, vs eps^-1 - 1 "
                f"{strict:.3e}, kappa {kappa:.3e} (tol {tol:.1e})")
            assert e <= tol, (path, method, iw, e)
    ctx.close()
