"""Device copies of the synthetic workloads (PyTorch tensors).

Z is generated on the GPU by synth/libsynth_gen.so from the same Philox
counters as the CPU generator (bit-identical values); energies, frequencies
and v^(1/2) are small and are copied from the CPU generator.  Input
generation only.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import c_int, c_uint32, c_void_p

import numpy as np

from .workloads import TAG_WC, TAG_Z, Workload, c3_word, z_scale_table

_LIB = None
_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth_gen.so")


def _lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} not built; run python -m paper_2506_03477_amd.build")
        lib = ctypes.CDLL(_LIB_PATH)
        lib.synth_z_fill.restype = c_int
        lib.synth_z_fill.argtypes = [c_void_p, c_int, c_int, c_int, c_int, c_uint32, c_uint32,
                                     c_void_p, c_void_p]
        lib.synth_wc_fill.restype = c_int
        lib.synth_wc_fill.argtypes = [c_void_p, c_int, c_int, c_uint32, c_uint32, c_void_p,
                                      c_void_p, c_void_p]
        _LIB = lib
    return _LIB


def z_block_device(wl: Workload, blk, device="cuda", scale_table=None, ztype=None):
    """Z of one block as a [nocc, nunocc, npb] complex device tensor."""
    import torch
    zt = ztype or wl.ztype
    dt = torch.complex128 if zt == "c128" else torch.complex64
    z = torch.empty((blk.nocc, blk.nunocc, wl.npb), dtype=dt, device=device)
    if z.numel() == 0:
        return z
    if scale_table is None:
        scale_table = torch.from_numpy(z_scale_table(wl.npb)).to(device)
    s = torch.cuda.current_stream(z.device)
    rc = _lib().synth_z_fill(c_void_p(z.data_ptr()), 1 if zt == "c64" else 0, wl.npb, blk.nocc,
                             blk.nunocc, blk.bid, c3_word(wl.cfg, TAG_Z, wl.seed),
                             c_void_p(scale_table.data_ptr()), c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"synth_z_fill failed ({rc})")
    return z


def device_workload(wl: Workload, q: int = 0, device="cuda", ztype=None, blocks=None):
    """(blocks, omega, vsqrt) for one q-point of a workload, on the device.
    blocks is a list of (z, eps_occ, eps_unocc, wk, Block) tuples."""
    import torch
    tab = torch.from_numpy(z_scale_table(wl.npb)).to(device)
    out = []
    for blk in (wl.blocks(q) if blocks is None else blocks):
        eo, eu = wl.energies(blk)
        z = z_block_device(wl, blk, device, tab, ztype)
        out.append((z, torch.from_numpy(eo).to(device), torch.from_numpy(eu).to(device),
                    blk.wk, blk))
    omega = torch.tensor(wl.omega, dtype=torch.float64, device=device)
    vsqrt = torch.from_numpy(wl.vsqrt()).to(device)
    return out, omega, vsqrt


def wc_block_device(wl: Workload, blk, device="cuda", tables=None):
    """Synthetic W^c of one block as a [nomega, nmu, nmu] complex128 device
    tensor (bit-identical to ``Workload.wc_block``)."""
    import torch
    nmu = blk.nunocc
    if tables is None:
        f2, c = wl.wc_tables(nmu)
        tables = (torch.from_numpy(f2).to(device), torch.from_numpy(np.ascontiguousarray(c)).to(device))
    w = torch.empty((wl.nomega, nmu, nmu), dtype=torch.complex128, device=device)
    s = torch.cuda.current_stream(w.device)
    rc = _lib().synth_wc_fill(c_void_p(w.data_ptr()), nmu, wl.nomega, blk.bid,
                              c3_word(wl.cfg, TAG_WC, wl.seed), c_void_p(tables[0].data_ptr()),
                              c_void_p(tables[1].data_ptr()), c_void_p(s.cuda_stream))
    if rc != 0:
        raise RuntimeError(f"synth_wc_fill failed ({rc})")
    return w


def device_sigc_workload(wl: Workload, q: int = 0, device="cuda", blocks=None):
    """Inputs of one q-point of a correlation workload on the device:
    (list of (z, wc, eps_mid (host numpy), wk, Block), eps_qp (host numpy))."""
    import torch
    tab = torch.from_numpy(z_scale_table(wl.npb)).to(device)
    wtab = {}
    out = []
    for blk in (wl.blocks(q) if blocks is None else blocks):
        if blk.nunocc not in wtab:
            f2, c = wl.wc_tables(blk.nunocc)
            wtab[blk.nunocc] = (torch.from_numpy(f2).to(device),
                                torch.from_numpy(np.ascontiguousarray(c)).to(device))
        z = z_block_device(wl, blk, device, tab, "c128")
        wc = wc_block_device(wl, blk, device, wtab[blk.nunocc])
        out.append((z, wc, wl.eps_mid(blk), blk.wk, blk))
    return out, wl.eps_qp(q)
