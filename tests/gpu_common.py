"""Helpers for the GPU parity tests: device problems from synthetic workloads
and the matching oracle results (oracle inputs come from synth/ only)."""
import numpy as np
import torch

import oracle
from paper_2506_03477_amd import Block, Problem
from synth.gpu import device_workload


def need_gpu():
    import pytest
    if not torch.cuda.is_available():
        pytest.skip("no GPU visible")


def device_problem(wl, q=0, ztype=None, blocks=None, device="cuda"):
    blks, omega, vsqrt = device_workload(wl, q, device, ztype=ztype, blocks=blocks)
    chi = torch.empty((wl.nomega, wl.npb, wl.npb), dtype=torch.complex128, device=device)
    prob = Problem([Block(z, eo, eu, wk) for z, eo, eu, wk, _ in blks], omega, chi)
    return prob, vsqrt, blks


def oracle_chi0(wl, q=0, ztype=None, blocks=None):
    w = wl if ztype is None else wl.replace(ztype=ztype)
    return oracle.chi0_workload(w, q, blocks)


def rel_fro(x, ref):
    return oracle.rel_fro(np.asarray(x), np.asarray(ref))


def assert_hermitian_exact(chi):
    c = chi if isinstance(chi, torch.Tensor) else torch.from_numpy(chi)
    assert torch.equal(c, c.conj().transpose(-1, -2))
    d = torch.diagonal(c, dim1=-2, dim2=-1)
    assert torch.all(d.imag == 0)


def host_blocks(blks, nocc_chunk, say=None, tag=""):
    """Oracle inputs streamed from device blocks (z, eps_occ, eps_unocc, wk,
    ...): chunks of `nocc_chunk` occupied states, Z copied to the host and
    upcast exactly to complex128.  The device Z comes from the synthetic
    generator, bit-identical to the CPU one."""
    for k, b in enumerate(blks):
        z, eo, eu, wk = b[0], b[1].cpu().numpy(), b[2].cpu().numpy(), b[3]
        if say is not None:
            say(f"{tag} block {k + 1}/{len(blks)}")
        for n0 in range(0, z.shape[0], nocc_chunk):
            n1 = min(z.shape[0], n0 + nocc_chunk)
            zc = z[n0:n1].cpu().numpy().astype(np.complex128)
            yield zc, eo[n0:n1], eu, wk
