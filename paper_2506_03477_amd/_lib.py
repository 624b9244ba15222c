"""ctypes binding of libchi0 (include/chi0.h).

Argument marshalling only: every step of the computation runs in the HIP
kernels of libchi0.so.  Tensors are PyTorch device tensors; the binding passes
their data pointers and the current HIP stream.  The library must have been
built (``python -m paper_2506_03477_amd.build``); importing this module fails
loudly otherwise, and there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_int, c_int32, c_int64, c_uint32, c_void_p
from dataclasses import dataclass
from typing import List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
# CHI0_LIB names another build of the same library (the host-sanitized build
# of build.build_host_sanitized()); by default the in-tree libchi0.so
LIB_PATH = os.environ.get("CHI0_LIB") or os.path.join(_HERE, "libchi0.so")

CHI0_OK = 0
CHI0_EINVAL = -1
CHI0_ENOMEM = -2
CHI0_EDEVICE = -3
CHI0_ENOTHPD = -4
CHI0_ESINGULAR = -5
CHI0_EUNSUPPORTED = -6

PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
ZTYPE = {"c128": 0, "c64": 1}
CHI0_ACCUMULATE = 1
CHI0_BF16_LOLO = 2
CHI0_USE_GRAPH = 4
CHI0_INV_GJ = 0
CHI0_INV_HPD = 1
CHI0_INV_HPD_FALLBACK_GJ = 2
INV_METHOD = {"gj": CHI0_INV_GJ, "hpd": CHI0_INV_HPD, "hpd_fallback_gj": CHI0_INV_HPD_FALLBACK_GJ}
CHI0_OUT_WC = 8
CHI0_NOALLOC_SCRATCH_BYTES = 256 << 20  # include/chi0.h


class chi0_block(ctypes.Structure):
    _fields_ = [("nocc", c_int32), ("nunocc", c_int32), ("z", c_void_p),
                ("eps_occ", c_void_p), ("eps_unocc", c_void_p), ("wk", c_double)]


class chi0_problem(ctypes.Structure):
    _fields_ = [("npb", c_int32), ("nblocks", c_int32), ("blocks", POINTER(chi0_block)),
                ("nomega", c_int32), ("omega", c_void_p), ("chi0", c_void_p)]


class sigx_block(ctypes.Structure):
    _fields_ = [("nocc", c_int32), ("nmu", c_int32), ("z", c_void_p), ("v", c_void_p),
                ("wk", c_double)]


class sigx_problem(ctypes.Structure):
    _fields_ = [("nqp", c_int32), ("nblocks", c_int32), ("blocks", POINTER(sigx_block)),
                ("sigx", c_void_p)]


class sigc_block(ctypes.Structure):
    _fields_ = [("nall", c_int32), ("nmu", c_int32), ("z", c_void_p), ("wc", c_void_p),
                ("eps_mid", c_void_p), ("wk", c_double)]


class sigc_problem(ctypes.Structure):
    _fields_ = [("nqp", c_int32), ("nblocks", c_int32), ("blocks", POINTER(sigc_block)),
                ("eps_qp", c_void_p), ("nomega", c_int32), ("pad", c_int32),
                ("omega", c_void_p), ("sigc", c_void_p)]


class chi0_hist(ctypes.Structure):
    _fields_ = [("nbins", c_int32), ("nreal", c_int32), ("edges", c_void_p), ("sigma", c_double),
                ("omega_re", c_void_p), ("chi0_re", c_void_p), ("hist", c_void_p)]


class Chi0Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libchi0 error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libchi0.so once (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built; run python -m paper_2506_03477_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp = c_void_p
    sig = {
        "chi0_version": (c_int, []),
        "chi0_status_string": (ctypes.c_char_p, [c_int]),
        "chi0_last_error": (ctypes.c_char_p, []),
        "chi0_create": (c_int, [POINTER(vp), c_int]),
        "chi0_destroy": (c_int, [vp]),
        "chi0_accumulate": (c_int, [vp, POINTER(chi0_problem), c_int32, c_int, c_int, c_double,
                                    c_uint32, vp]),
        "dielectric_invert": (c_int, [vp, c_int32, c_int32, vp, vp, vp, vp, vp, c_uint32, vp]),
        "dielectric_invert_noalloc": (c_int, [vp, c_int32, c_int32, vp, vp, vp, vp, vp, c_uint32, vp]),
        "chi0_sync": (c_int, [vp]),
        "sigx_accumulate": (c_int, [vp, POINTER(sigx_problem), c_int32, c_int, c_int, c_uint32, vp]),
        "sigc_accumulate": (c_int, [vp, POINTER(sigc_problem), c_int32, c_int, c_int, c_uint32, vp]),
        "chi0_hist_accumulate": (c_int, [vp, POINTER(chi0_problem), POINTER(chi0_hist), c_int32, c_int,
                                         c_int, c_double, c_uint32, vp]),
        "sigc_set_variant": (c_int, [vp, c_int32]),
        "chi0_hist_stats": (c_int, [vp, POINTER(c_int64), POINTER(c_int32)]),
        "sigc_set_workspace_cap": (c_int, [vp, c_int64]),
        "chi0_set_partial_cap": (c_int, [vp, c_int64]),
        "chi0_tile_count": (c_int, [c_int]),
        "chi0_tile_info": (c_int, [c_int, c_int32, POINTER(c_int32), POINTER(c_int32),
                                   POINTER(c_int32), POINTER(c_int32)]),
        "chi0_set_tile": (c_int, [vp, c_int, c_int32]),
        "chi0_set_flush": (c_int, [vp, c_int32]),
        "chi0_get_tile": (c_int, [vp, c_int, POINTER(c_int32)]),
        "chi0_last_tile": (c_int, [vp, c_int, POINTER(c_int32)]),
        "chi0_tile_choice": (c_int, [c_int, POINTER(chi0_problem), c_int32, POINTER(c_int32)]),
        "chi0_tile_lists": (c_int, [c_int, c_int32]),
        "chi0_tile_diag_skip": (c_int, [c_int, c_int32]),
        "chi0_set_xcd_slack": (c_int, [vp, c_int32]),
        "chi0_autotune": (c_int, [vp, POINTER(chi0_problem), c_int32, c_int, c_int, c_double,
                                  c_int32, POINTER(c_int32), POINTER(c_double), vp]),
        "chi0_plan_inspect": (c_int, [POINTER(chi0_problem), c_int32, c_int, c_int32, c_int32,
                                      POINTER(c_int32), POINTER(c_int32), POINTER(c_int32),
                                      c_int32, POINTER(c_double), POINTER(c_double)]),
        "chi0_profile_enable": (c_int, [vp, c_int]),
        "chi0_profile_read": (c_int, [vp, POINTER(c_double), POINTER(c_int64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _check(rc: int) -> int:
    if rc < 0:
        lib = load()
        raise Chi0Error(rc, lib.chi0_last_error().decode() or lib.chi0_status_string(rc).decode())
    return rc


def _stream_ptr(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype=None, what="tensor"):
    import torch
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{what} must be {dtype}, got {t.dtype}")
    return c_void_p(t.data_ptr())


@dataclass
class Block:
    """One k-point (x spin) block: z [nocc, nunocc, npb] complex device tensor,
    eps_occ [nocc] / eps_unocc [nunocc] float64 device tensors, weight wk."""
    z: object
    eps_occ: object
    eps_unocc: object
    wk: float


@dataclass
class Problem:
    """One q-point: blocks, omega [nomega] float64 device tensor, chi0 output
    [nomega, npb, npb] complex128 device tensor."""
    blocks: List[Block]
    omega: object
    chi0: object

    @property
    def npb(self) -> int:
        return int(self.chi0.shape[-1])


@dataclass
class SigxBlock:
    """One k-point of the exchange self-energy: z [nocc, nmu, nqp] complex
    device tensor, v [nmu] float64 device tensor (Coulomb eigenvalues), wk."""
    z: object
    v: object
    wk: float


@dataclass
class SigxProblem:
    """One q-point: blocks and the [nqp, nqp] complex128 output."""
    blocks: List[SigxBlock]
    sigx: object

    @property
    def nqp(self) -> int:
        return int(self.sigx.shape[-1])


def _marshal_sigx(problems: Sequence[SigxProblem]):
    import torch
    keep = []
    arr = (sigx_problem * len(problems))()
    for i, p in enumerate(problems):
        nqp, nqp2 = p.sigx.shape
        if nqp != nqp2:
            raise ValueError("sigx must be [nqp, nqp]")
        barr = (sigx_block * max(1, len(p.blocks)))()
        for j, b in enumerate(p.blocks):
            nmu = int(b.v.numel())
            has_z = b.z is not None and b.z.numel() > 0
            nocc = int(b.z.shape[0]) if has_z else 0
            if has_z and tuple(b.z.shape) != (nocc, nmu, nqp):
                raise ValueError(f"block {j}: z shape {tuple(b.z.shape)} != {(nocc, nmu, nqp)}")
            barr[j].nocc = nocc
            barr[j].nmu = nmu
            barr[j].z = _dev_ptr(b.z, what="z") if has_z else None
            barr[j].v = _dev_ptr(b.v, torch.float64, "v") if nmu else None
            barr[j].wk = float(b.wk)
        keep.append(barr)
        arr[i].nqp = nqp
        arr[i].nblocks = len(p.blocks)
        arr[i].blocks = ctypes.cast(barr, POINTER(sigx_block))
        arr[i].sigx = _dev_ptr(p.sigx, torch.complex128, "sigx")
    return arr, keep


@dataclass
class HistSpec:
    """Histogram route settings of one problem: bin edges (host, > 0,
    increasing), spread sigma, optional real frequencies (host) with their
    [nreal, npb, npb] complex128 device output, optional [nbins, npb, npb]
    complex128 device output of the bin matrices."""
    edges: object
    sigma: float = 0.0
    omega_re: object = None
    chi0_re: object = None
    hist: object = None


@dataclass
class SigcBlock:
    """One k-point of the imaginary-axis correlation self-energy: z
    [nall, nmu, nqp] and wc [nomega, nmu, nmu] complex128 device tensors,
    eps_mid [nall] host float64 array (energies of the intermediate states),
    wk."""
    z: object
    wc: object
    eps_mid: object
    wk: float


@dataclass
class SigcProblem:
    """One q-point: blocks, host eps_qp [nqp] and omega [nomega] (float64),
    and the [nqp, nqp] complex128 device output."""
    blocks: List[SigcBlock]
    eps_qp: object
    omega: object
    sigc: object


def _host_f64(x, n, what):
    import numpy as np
    a = np.ascontiguousarray(np.asarray(x.cpu() if hasattr(x, "cpu") else x, dtype=np.float64))
    if a.ndim != 1 or a.size != n:
        raise ValueError(f"{what} must have {n} values, has shape {a.shape}")
    return a


def _marshal_sigc(problems: Sequence[SigcProblem]):
    import torch
    keep = []
    arr = (sigc_problem * len(problems))()
    for i, p in enumerate(problems):
        nqp, nqp2 = p.sigc.shape
        if nqp != nqp2:
            raise ValueError("sigc must be [nqp, nqp]")
        eq = _host_f64(p.eps_qp, nqp, "eps_qp")
        om = _host_f64(p.omega, len(p.omega), "omega")
        nomega = om.size
        barr = (sigc_block * max(1, len(p.blocks)))()
        for j, b in enumerate(p.blocks):
            nomega_b, nmu, nmu2 = b.wc.shape
            if nmu != nmu2 or nomega_b != nomega:
                raise ValueError(f"block {j}: wc shape {tuple(b.wc.shape)} != {(nomega, nmu, nmu)}")
            has_z = b.z is not None and b.z.numel() > 0
            nall = int(b.z.shape[0]) if has_z else 0
            if has_z and tuple(b.z.shape) != (nall, nmu, nqp):
                raise ValueError(f"block {j}: z shape {tuple(b.z.shape)} != {(nall, nmu, nqp)}")
            em = _host_f64(b.eps_mid, nall, "eps_mid")
            keep.append(em)
            barr[j].nall = nall
            barr[j].nmu = nmu
            barr[j].z = _dev_ptr(b.z, torch.complex128, "z") if has_z else None
            barr[j].wc = _dev_ptr(b.wc, torch.complex128, "wc")
            barr[j].eps_mid = em.ctypes.data if nall else None
            barr[j].wk = float(b.wk)
        keep += [barr, eq, om]
        arr[i].nqp = nqp
        arr[i].nblocks = len(p.blocks)
        arr[i].blocks = ctypes.cast(barr, POINTER(sigc_block))
        arr[i].eps_qp = eq.ctypes.data
        arr[i].nomega = nomega
        arr[i].pad = 0
        arr[i].omega = om.ctypes.data
        arr[i].sigc = _dev_ptr(p.sigc, torch.complex128, "sigc")
    return arr, keep


def _marshal(problems: Sequence[Problem]):
    import torch
    keep = []
    arr = (chi0_problem * len(problems))()
    for i, p in enumerate(problems):
        nomega, npb, npb2 = p.chi0.shape
        if npb != npb2 or p.omega.numel() != nomega:
            raise ValueError("chi0 must be [nomega, npb, npb] with omega [nomega]")
        barr = (chi0_block * max(1, len(p.blocks)))()
        for j, b in enumerate(p.blocks):
            nocc, nunocc = int(b.eps_occ.numel()), int(b.eps_unocc.numel())
            if b.z is not None and b.z.numel():
                if tuple(b.z.shape) != (nocc, nunocc, npb):
                    raise ValueError(f"block {j}: z shape {tuple(b.z.shape)} != {(nocc, nunocc, npb)}")
            barr[j].nocc = nocc
            barr[j].nunocc = nunocc
            barr[j].z = _dev_ptr(b.z, what="z") if b.z is not None and b.z.numel() else None
            barr[j].eps_occ = _dev_ptr(b.eps_occ, torch.float64, "eps_occ") if nocc else None
            barr[j].eps_unocc = _dev_ptr(b.eps_unocc, torch.float64, "eps_unocc") if nunocc else None
            barr[j].wk = float(b.wk)
        keep.append(barr)
        arr[i].npb = npb
        arr[i].nblocks = len(p.blocks)
        arr[i].blocks = ctypes.cast(barr, POINTER(chi0_block))
        arr[i].nomega = nomega
        arr[i].omega = _dev_ptr(p.omega, torch.float64, "omega")
        arr[i].chi0 = _dev_ptr(p.chi0, torch.complex128, "chi0")
    return arr, keep


def tile_choice(precision: str, shapes) -> int:
    """The tile configuration the library's cost model picks for problems of
    the given shapes when no tile is fixed or tuned (host computation, no
    device).  shapes: [(npb, nomega, [(nocc, nunocc), ...]), ...]."""
    lib = load()
    keep = []
    arr = (chi0_problem * max(1, len(shapes)))()
    for i, (npb, nomega, blocks) in enumerate(shapes):
        barr = (chi0_block * max(1, len(blocks)))()
        for j, (nocc, nunocc) in enumerate(blocks):
            barr[j].nocc = int(nocc)
            barr[j].nunocc = int(nunocc)
            barr[j].z = barr[j].eps_occ = barr[j].eps_unocc = None
            barr[j].wk = 1.0
        keep.append(barr)
        arr[i].npb = int(npb)
        arr[i].nblocks = len(blocks)
        arr[i].blocks = ctypes.cast(barr, POINTER(chi0_block))
        arr[i].nomega = int(nomega)
        arr[i].omega = None
        arr[i].chi0 = None
    t = c_int32(-1)
    _check(lib.chi0_tile_choice(PREC[precision], arr, len(shapes), byref(t)))
    return t.value


def _ztype_of(problems: Sequence[Problem], precision: str) -> int:
    """The Z type of the call: that of the blocks' Z data; without any (every
    block empty), the dtype of an empty Z tensor, else the precision's own
    (complex128 for FP64, complex64 otherwise)."""
    import torch
    hint = None
    for p in problems:
        for b in p.blocks:
            if b.z is not None:
                zt = ZTYPE["c128"] if b.z.dtype == torch.complex128 else ZTYPE["c64"]
                if b.z.numel():
                    return zt
                hint = zt if hint is None else hint
    if hint is not None:
        return hint
    return ZTYPE["c128"] if precision == "fp64" else ZTYPE["c64"]


class Context:
    """A libchi0 handle on one GPU."""

    def __init__(self, device: int = 0):
        self._lib = load()
        self._h = c_void_p()
        _check(self._lib.chi0_create(byref(self._h), int(device)))

    def close(self):
        if self._h:
            self._lib.chi0_destroy(self._h)
            self._h = c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- chi0 ---------------------------------------------------------------
    def chi0_accumulate(self, problems: Sequence[Problem], precision: str = "fp64",
                        delta_min: float = 0.0, accumulate: bool = False,
                        lolo: bool = False, graph: bool = False, stream=None) -> None:
        arr, keep = _marshal(problems)
        flags = (CHI0_ACCUMULATE if accumulate else 0) | (CHI0_BF16_LOLO if lolo else 0) | \
            (CHI0_USE_GRAPH if graph else 0)
        _check(self._lib.chi0_accumulate(self._h, arr, len(problems), _ztype_of(problems, precision),
                                         PREC[precision], float(delta_min), flags,
                                         _stream_ptr(stream)))

    # -- exchange self-energy --------------------------------------------------
    def sigx_accumulate(self, problems: Sequence[SigxProblem], precision: str = "fp64",
                        accumulate: bool = False, lolo: bool = False, graph: bool = False,
                        stream=None) -> None:
        arr, keep = _marshal_sigx(problems)
        zt = _ztype_of(problems, precision)
        flags = (CHI0_ACCUMULATE if accumulate else 0) | (CHI0_BF16_LOLO if lolo else 0) | \
            (CHI0_USE_GRAPH if graph else 0)
        _check(self._lib.sigx_accumulate(self._h, arr, len(problems), zt, PREC[precision], flags,
                                         _stream_ptr(stream)))

    # -- histogram route ---------------------------------------------------------
    def chi0_hist_accumulate(self, problems: Sequence[Problem], hists: Sequence["HistSpec"],
                             precision: str = "fp64", delta_min: float = 0.0, lolo: bool = False,
                             stream=None) -> None:
        import numpy as np
        import torch
        if len(hists) != len(problems):
            raise ValueError("one HistSpec per problem")
        arr, keep = _marshal(problems)
        harr = (chi0_hist * max(1, len(hists)))()
        for i, (p, hs) in enumerate(zip(problems, hists)):
            npb = int(p.chi0.shape[-1])
            e = np.ascontiguousarray(np.asarray(hs.edges, dtype=np.float64))
            wr = np.ascontiguousarray(np.asarray(hs.omega_re if hs.omega_re is not None else [],
                                                 dtype=np.float64))
            keep += [e, wr]
            harr[i].nbins = e.size - 1
            harr[i].nreal = wr.size
            harr[i].edges = e.ctypes.data
            harr[i].sigma = float(hs.sigma)
            harr[i].omega_re = wr.ctypes.data if wr.size else None
            if wr.size:
                if tuple(hs.chi0_re.shape) != (wr.size, npb, npb):
                    raise ValueError("chi0_re must be [nreal, npb, npb]")
                harr[i].chi0_re = _dev_ptr(hs.chi0_re, torch.complex128, "chi0_re")
            else:
                harr[i].chi0_re = None
            if hs.hist is not None:
                if tuple(hs.hist.shape) != (e.size - 1, npb, npb):
                    raise ValueError("hist must be [nbins, npb, npb]")
                harr[i].hist = _dev_ptr(hs.hist, torch.complex128, "hist")
            else:
                harr[i].hist = None
        flags = CHI0_BF16_LOLO if lolo else 0
        _check(self._lib.chi0_hist_accumulate(self._h, arr, harr, len(problems), _ztype_of(problems, precision),
                                              PREC[precision], float(delta_min), flags,
                                              _stream_ptr(stream)))

    def hist_stats(self):
        """(records kept, bins used) of the last chi0_hist_accumulate call."""
        r, b = c_int64(), c_int32()
        _check(self._lib.chi0_hist_stats(self._h, byref(r), byref(b)))
        return int(r.value), int(b.value)

    # -- imaginary-axis correlation self-energy --------------------------------
    def sigc_accumulate(self, problems: Sequence[SigcProblem], precision: str = "fp64",
                        accumulate: bool = False, stream=None) -> None:
        arr, keep = _marshal_sigc(problems)
        flags = CHI0_ACCUMULATE if accumulate else 0
        _check(self._lib.sigc_accumulate(self._h, arr, len(problems), ZTYPE["c128"],
                                         PREC[precision], flags, _stream_ptr(stream)))

    def sigc_set_variant(self, variant: int) -> None:
        _check(self._lib.sigc_set_variant(self._h, int(variant)))

    def sigc_set_workspace_cap(self, nbytes: int) -> None:
        _check(self._lib.sigc_set_workspace_cap(self._h, int(nbytes)))

    def set_partial_cap(self, nbytes: int) -> None:
        """Bytes of FP64 partial tiles one rank-K launch may use (0: default)."""
        _check(self._lib.chi0_set_partial_cap(self._h, int(nbytes)))

    # -- dielectric ----------------------------------------------------------
    def dielectric_invert(self, vsqrt, chi0, eps_inv, eps=None, wc=None, method: str = "gj",
                          stream=None) -> None:
        import torch
        nomega, npb, _ = chi0.shape
        flags = (CHI0_OUT_WC if wc is not None else 0) | INV_METHOD[method]
        _check(self._lib.dielectric_invert(
            self._h, npb, nomega, _dev_ptr(vsqrt, torch.float64, "vsqrt"),
            _dev_ptr(chi0, torch.complex128, "chi0"), _dev_ptr(eps, torch.complex128, "eps"),
            _dev_ptr(eps_inv, torch.complex128, "eps_inv"), _dev_ptr(wc, torch.complex128, "wc"),
            flags, _stream_ptr(stream)))

    def dielectric_invert_noalloc(self, vsqrt, chi0, eps_inv, eps=None, wc=None,
                                  method: str = "gj", stream=None) -> None:
        """dielectric_invert with its workspace in the library's fixed
        device array (no allocation); see CHI0_NOALLOC_SCRATCH_BYTES."""
        import torch
        nomega, npb, _ = chi0.shape
        flags = (CHI0_OUT_WC if wc is not None else 0) | INV_METHOD[method]
        _check(self._lib.dielectric_invert_noalloc(
            self._h, npb, nomega, _dev_ptr(vsqrt, torch.float64, "vsqrt"),
            _dev_ptr(chi0, torch.complex128, "chi0"), _dev_ptr(eps, torch.complex128, "eps"),
            _dev_ptr(eps_inv, torch.complex128, "eps_inv"), _dev_ptr(wc, torch.complex128, "wc"),
            flags, _stream_ptr(stream)))

    def sync(self) -> None:
        _check(self._lib.chi0_sync(self._h))

    # -- tiles / tuning / timing -----------------------------------------------
    def tile_count(self, precision: str) -> int:
        return _check(self._lib.chi0_tile_count(PREC[precision]))

    def tile_info(self, precision: str, tile: int):
        a, b, c, d = c_int32(), c_int32(), c_int32(), c_int32()
        _check(self._lib.chi0_tile_info(PREC[precision], tile, byref(a), byref(b), byref(c), byref(d)))
        return {"tile_p": a.value, "tile_q": b.value, "kchunk": c.value, "flush_len": d.value}

    def tile_lists(self, precision: str, tile: int) -> int:
        """Work lists per workgroup of a tile configuration (1 or 4)."""
        return _check(self._lib.chi0_tile_lists(PREC[precision], tile))

    def tile_diag_skip(self, precision: str, tile: int) -> bool:
        """True when the configuration leaves out the 32 x 32 blocks of
        diagonal tiles that lie entirely above the diagonal."""
        return bool(_check(self._lib.chi0_tile_diag_skip(PREC[precision], tile)))

    def set_tile(self, precision: str, tile: int) -> None:
        _check(self._lib.chi0_set_tile(self._h, PREC[precision], tile))

    def set_xcd_slack(self, stages: int) -> None:
        """XCD lockstep slack in stages (-1 default, 0 off, -2 unmeetable)."""
        _check(self._lib.chi0_set_xcd_slack(self._h, int(stages)))

    def set_flush(self, pairs: int) -> None:
        _check(self._lib.chi0_set_flush(self._h, int(pairs)))

    def get_tile(self, precision: str) -> int:
        t = c_int32()
        _check(self._lib.chi0_get_tile(self._h, PREC[precision], byref(t)))
        return t.value

    def last_tile(self, precision: str) -> int:
        """Configuration of this handle's last rank-K launch at `precision`
        (-1 before the first)."""
        t = c_int32(-1)
        _check(self._lib.chi0_last_tile(self._h, PREC[precision], byref(t)))
        return t.value

    def autotune(self, problems: Sequence[Problem], precision: str, delta_min: float = 0.0,
                 reps: int = 2, stream=None):
        arr, keep = _marshal(problems)
        n = self.tile_count(precision)
        ms = (c_double * max(1, n))()
        best = c_int32()
        _check(self._lib.chi0_autotune(self._h, arr, len(problems), _ztype_of(problems, precision),
                                       PREC[precision], float(delta_min), reps, byref(best), ms,
                                       _stream_ptr(stream)))
        return best.value, [ms[i] for i in range(n)]

    def profile_enable(self, on: bool = True) -> None:
        _check(self._lib.chi0_profile_enable(self._h, 1 if on else 0))

    def profile_read(self):
        ms, n = c_double(), c_int64()
        _check(self._lib.chi0_profile_read(self._h, byref(ms), byref(n)))
        return ms.value, n.value


def header_functions() -> List[str]:
    """Names of the functions declared in include/chi0.h."""
    import re
    hdr = os.path.join(os.path.dirname(_HERE), "include", "chi0.h")
    with open(hdr) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w[\w\s\*]*?\b(\w+)\s*\(", src, flags=re.M)))
