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
