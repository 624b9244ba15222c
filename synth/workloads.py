"""Seeded synthetic workloads for the chi0 + dielectric hot path.

This module generates inputs only: product-basis matrix elements Z, band
energies, imaginary frequencies, the Coulomb square roots and the block
layout (k-points x spins, with their occupied / unoccupied counts).  It holds
none of the polarization arithmetic and is shared, read-only, by the CPU
oracle and by the GPU path.

Inputs stand in for the paper's ecalj runs on (InAs)n(GaSb)n superlattices
and Ni2MnGa (Table "systemsize"), which are not available: shapes follow the
paper's size parameters (Table "computationalcost"), values are synthetic.

Every random value is a pure function of a Philox4x32-10 counter, so any
element of any block can be regenerated on its own (the oracle uses this to
check sampled entries of full-size runs) and the GPU generator in
``synth/csrc/synth_gen.hip`` reproduces the CPU values bit for bit.

Counter layout (c0, c1, c2, c3), key (2506, 3477):
  c0, c1 : low / high 32 bits of the element index inside its stream
  c2     : block id = (q * nspin + spin) * nk + k
  c3     : tag | cfg << 8 | seed << 16, tag in {Z, occupied energy,
           unoccupied energy, block size}

Z_{n n'}(I), complex, for pair (n, n') and product-basis index I:
  e = (n * nunocc + n') * npb + I,   (r0, r1, r2, r3) = philox(e, ...)
  re = (sum of the four 16-bit halves of r0, r1 - 131070) * F[I]
  im = (sum of the four 16-bit halves of r2, r3 - 131070) * F[I]
  F[I] = sqrt(3) / 65536 * exp(-I / 32)
The centred sum of four uniform 16-bit integers has unit variance after the
sqrt(3)/65536 scale (an Irwin-Hall approximation of a standard normal); the
exp(-I/32) factor imposes the decay along the product-basis index.  Complex64
inputs are the complex128 values rounded to nearest.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple, Union

import numpy as np

from .philox import philox4x32

KEY0 = 2506
KEY1 = 3477
TAG_Z = 0
TAG_EOCC = 1
TAG_EUNOCC = 2
TAG_SIZE = 3
TAG_EQP = 4
TAG_WC = 5

IRWIN_HALL_CENTRE = 131070  # 4 * (65535 / 2)


def c3_word(cfg: int, tag: int, seed: int = 0) -> int:
    return (tag & 0xFF) | ((cfg & 0xFF) << 8) | ((seed & 0xFFFF) << 16)


def z_scale_table(npb: int) -> np.ndarray:
    """F[I] = sqrt(3)/65536 * exp(-I/32), float64, I = 0..npb-1."""
    idx = np.arange(npb, dtype=np.float64)
    return (math.sqrt(3.0) / 65536.0) * np.exp(-idx / 32.0)


def _halves_sum(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    m = np.uint64(0xFFFF)
    s16 = np.uint64(16)
    return (a & m) + (a >> s16) + (b & m) + (b >> s16)


def gauss_legendre_imag_axis(n: int, omega_c: float = 1.0) -> np.ndarray:
    """n Gauss-Legendre nodes x on (-1, 1) mapped to [0, inf) by
    omega = omega_c (1 + x) / (1 - x), ascending (Hartree)."""
    x, _ = np.polynomial.legendre.leggauss(n)
    return np.sort(omega_c * (1.0 + x) / (1.0 - x))


def hist_edges(emax: float, e0: float = 5e-6, ratio: float = 1.03) -> np.ndarray:
    """Histogram bin edges of the paper's real-axis mesh, e0 * ratio^j Ha
    (1e-5 * 1.03^j Ry), from e0 to the first edge above emax."""
    n = int(math.ceil(math.log(emax / e0) / math.log(ratio))) + 1
    return e0 * ratio ** np.arange(n + 1, dtype=np.float64)


def vsqrt_table(npb: int) -> np.ndarray:
    """Square roots of the Coulomb eigenvalues, s_I = 1 / (1 + I)."""
    return 1.0 / (1.0 + np.arange(npb, dtype=np.float64))


@dataclass(frozen=True)
class Block:
    """One k-point (x spin) block of one q-point."""
    q: int
    spin: int
    k: int
    nocc: int
    nunocc: int
    wk: float
    bid: int

    @property
    def npairs(self) -> int:
        return self.nocc * self.nunocc


IntSpec = Union[int, Tuple[int, int]]


@dataclass(frozen=True)
class Workload:
    name: str
    cfg: int
    npb: int
    nq: int
    nspin: int
    nk: int
    nocc: IntSpec
    nunocc: IntSpec
    omega: Tuple[float, ...]
    ztype: str                     # "c128" or "c64"
    delta_min: float = 0.0
    occ_range: Tuple[float, float] = (-0.8, 0.0)
    unocc_range: Tuple[float, float] = (0.05, 3.0)
    metallic: bool = False
    seed: int = 0
    paths: Tuple[str, ...] = ("fp64",)
    nval: int = 0                  # correlation workloads: occupied states among n', n

    # ------------------------------------------------------------------ layout
    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)

    @property
    def nomega(self) -> int:
        return len(self.omega)

    def omega_array(self) -> np.ndarray:
        return np.asarray(self.omega, dtype=np.float64)

    def vsqrt(self) -> np.ndarray:
        return vsqrt_table(self.npb)

    def _size(self, spec: IntSpec, bid: int, word: int) -> int:
        if isinstance(spec, int):
            return spec
        lo, hi = spec
        r = philox4x32(bid, 0, bid, c3_word(self.cfg, TAG_SIZE, self.seed), KEY0, KEY1)
        u = int(r[word])
        return lo + ((u * (hi - lo + 1)) >> 32)

    def blocks(self, q: int = 0) -> List[Block]:
        out = []
        wk = 1.0 / self.nk
        for spin in range(self.nspin):
            for k in range(self.nk):
                bid = (q * self.nspin + spin) * self.nk + k
                out.append(Block(q=q, spin=spin, k=k,
                                 nocc=self._size(self.nocc, bid, 0),
                                 nunocc=self._size(self.nunocc, bid, 1),
                                 wk=wk, bid=bid))
        return out

    def npairs(self, q: int = 0) -> int:
        return sum(b.npairs for b in self.blocks(q))

    # ---------------------------------------------------------------- energies
    def _uniform(self, n: int, bid: int, tag: int, offset: int = 0) -> np.ndarray:
        idx = np.arange(offset, offset + n, dtype=np.uint64)
        r = philox4x32(idx, 0, bid, c3_word(self.cfg, tag, self.seed), KEY0, KEY1)
        return r[0].astype(np.float64) * 2.0 ** -32

    def energies(self, blk: Block) -> Tuple[np.ndarray, np.ndarray]:
        """(eps_occ[nocc] at k, eps_unocc[nunocc] at k+q), float64, sorted."""
        olo, ohi = self.occ_range
        ulo, uhi = self.unocc_range
        if not self.metallic:
            eo = olo + (ohi - olo) * self._uniform(blk.nocc, blk.bid, TAG_EOCC)
            eu = ulo + (uhi - ulo) * self._uniform(blk.nunocc, blk.bid, TAG_EUNOCC)
        else:
            # Metallic cell with E_F = 0: four occupied and four unoccupied
            # states per block are planted within 2e-4 Ha of E_F, so that a
            # few pairs fall below the intraband cut delta_min.
            nf_o = min(4, blk.nocc)
            nf_u = min(4, blk.nunocc)
            uo = self._uniform(blk.nocc, blk.bid, TAG_EOCC)
            uu = self._uniform(blk.nunocc, blk.bid, TAG_EUNOCC)
            eo = np.concatenate([olo + (ohi - olo) * uo[: blk.nocc - nf_o],
                                 -2e-4 + 2e-4 * uo[blk.nocc - nf_o:]])
            eu = np.concatenate([2e-4 * uu[:nf_u],
                                 ulo + (uhi - ulo) * uu[nf_u:]])
        return np.sort(eo), np.sort(eu)

    def coulomb(self, blk: Block) -> np.ndarray:
        """Coulomb eigenvalues for the exchange workloads (whose blocks have
        nunocc = number of product-basis functions mu): v_mu = (1 + mu)^(-2/3),
        the 1/|G|^2 decay of plane-wave-like functions ordered by |G|, with
        |G|^2 growing as mu^(2/3)."""
        return (1.0 + np.arange(blk.nunocc, dtype=np.float64)) ** (-2.0 / 3.0)

    # ---------------------------------------- correlation self-energy inputs
    # For the correlation workloads the block fields read: npb = nqp (the
    # quasiparticle states n, innermost index of Z), nocc = nall (all
    # intermediate states n'), nunocc = number of product-basis functions mu.
    def eps_qp(self, q: int = 0) -> np.ndarray:
        """Quasiparticle energies eps_{q n}, n < npb: the lowest nval
        occupied in occ_range, the rest unoccupied in unocc_range, sorted."""
        nv = min(self.nval, self.npb)
        bid = 0xFFFF0000 | (q & 0xFFFF)
        u = self._uniform(self.npb, bid, TAG_EQP)
        olo, ohi = self.occ_range
        ulo, uhi = self.unocc_range
        e = np.concatenate([olo + (ohi - olo) * u[:nv], ulo + (uhi - ulo) * u[nv:]])
        return np.sort(e)

    def eps_mid(self, blk: Block) -> np.ndarray:
        """Intermediate-state energies eps_{q-k, n'}, n' < nocc (= nall):
        nval occupied, the rest unoccupied, sorted."""
        nv = min(self.nval, blk.nocc)
        olo, ohi = self.occ_range
        ulo, uhi = self.unocc_range
        eo = olo + (ohi - olo) * self._uniform(nv, blk.bid, TAG_EOCC)
        eu = ulo + (uhi - ulo) * self._uniform(blk.nocc - nv, blk.bid, TAG_EUNOCC)
        return np.sort(np.concatenate([eo, eu]))

    def wc_tables(self, nmu: int) -> Tuple[np.ndarray, np.ndarray]:
        """Factor tables of the synthetic W^c (see ``wc_block``):
        F2[d] = 0.02 sqrt(3)/65536 exp(-d/8) for d = |mu - nu|, and
        C[i][mu] = s_mu / sqrt(1 + (w_i / Omega_mu)^2) with s_mu = 1/(1+mu),
        Omega_mu = 0.3 + 3 mu / nmu (Hartree)."""
        d = np.arange(nmu, dtype=np.float64)
        f2 = (0.02 * math.sqrt(3.0) / 65536.0) * np.exp(-d / 8.0)
        om = self.omega_array()[:, None]
        big_omega = 0.3 + 3.0 * d / max(nmu, 1)
        c = (1.0 / (1.0 + d))[None, :] / np.sqrt(1.0 + (om / big_omega[None, :]) ** 2)
        return f2, c

    def wc_block(self, blk: Block, tables=None) -> np.ndarray:
        """Synthetic correlation interaction W^c_k(i w_i)[mu][nu], complex128
        [nomega][nmu][nmu] with nmu = blk.nunocc: Hermitian and negative
        definite at every w_i, decaying as 1/w^2.  W = -(C_i[mu] C_i[nu]) h,
        with h[mu][mu] = 1 and, for mu > nu, h = x F2[mu - nu] where x is the
        Irwin-Hall complex draw at element e = mu * nmu + nu of stream
        TAG_WC; h[nu][mu] = conj(h[mu][nu]).  Every value is one or two
        correctly rounded products of exact numbers, so the GPU generator
        reproduces it bit for bit."""
        nmu = blk.nunocc
        f2, c = self.wc_tables(nmu) if tables is None else tables
        mu = np.arange(nmu, dtype=np.uint64)
        e = (mu[:, None] * np.uint64(nmu) + mu[None, :]).reshape(-1)
        r0, r1, r2, r3 = philox4x32(e & np.uint64(0xFFFFFFFF), e >> np.uint64(32), blk.bid,
                                    c3_word(self.cfg, TAG_WC, self.seed), KEY0, KEY1)
        xr = (_halves_sum(r0, r1).astype(np.int64) - IRWIN_HALL_CENTRE).astype(np.float64)
        xi = (_halves_sum(r2, r3).astype(np.int64) - IRWIN_HALL_CENTRE).astype(np.float64)
        xr = xr.reshape(nmu, nmu)
        xi = xi.reshape(nmu, nmu)
        dd = np.abs(np.arange(nmu)[:, None] - np.arange(nmu)[None, :])
        lower = np.tril(np.ones((nmu, nmu), bool), -1)
        hr = np.where(lower, xr * f2[dd], 0.0)
        hi = np.where(lower, xi * f2[dd], 0.0)
        hr = hr + hr.T + np.eye(nmu)
        hi = hi - hi.T
        out = np.empty((self.nomega, nmu, nmu), np.complex128)
        for i in range(self.nomega):
            cc = c[i][:, None] * c[i][None, :]
            out[i].real = -(cc * hr)
            out[i].imag = -(cc * hi)
        return out

    # ----------------------------------------------------------------------- Z
    def z_elements(self, blk: Block, pair_index: np.ndarray,
                   cols: np.ndarray) -> np.ndarray:
        """Z for pairs ``pair_index`` (= n * nunocc + n') and basis indices
        ``cols``; returns complex128 of shape (len(pair_index), len(cols)),
        or complex64-rounded values upcast when ztype is c64."""
        pair_index = np.asarray(pair_index, dtype=np.uint64).reshape(-1, 1)
        cols_u = np.asarray(cols, dtype=np.uint64).reshape(1, -1)
        e = pair_index * np.uint64(self.npb) + cols_u
        r0, r1, r2, r3 = philox4x32(e & np.uint64(0xFFFFFFFF), e >> np.uint64(32),
                                    blk.bid, c3_word(self.cfg, TAG_Z, self.seed),
                                    KEY0, KEY1)
        f = z_scale_table(self.npb)[np.asarray(cols, dtype=np.int64)].reshape(1, -1)
        re = (_halves_sum(r0, r1).astype(np.int64) - IRWIN_HALL_CENTRE).astype(np.float64) * f
        im = (_halves_sum(r2, r3).astype(np.int64) - IRWIN_HALL_CENTRE).astype(np.float64) * f
        if self.ztype == "c64":
            re = re.astype(np.float32).astype(np.float64)
            im = im.astype(np.float32).astype(np.float64)
        return re + 1j * im

    def z_block(self, blk: Block, chunk_pairs: int = 4096) -> np.ndarray:
        """Full Z for a block as (nocc, nunocc, npb), complex128 (c128
        workloads) or complex64 (c64 workloads)."""
        dt = np.complex128 if self.ztype == "c128" else np.complex64
        out = np.empty((blk.nocc * blk.nunocc, self.npb), dtype=dt)
        cols = np.arange(self.npb)
        step = max(1, chunk_pairs * 64 // max(self.npb, 1))
        for p0 in range(0, blk.npairs, step):
            p1 = min(blk.npairs, p0 + step)
            out[p0:p1] = self.z_elements(blk, np.arange(p0, p1), cols)
        return out.reshape(blk.nocc, blk.nunocc, self.npb)


# --------------------------------------------------------------------------
# The five workloads.  Sizes and ranges follow the problem statement; where it
# is silent the choice is stated here (and in the design notes).
# --------------------------------------------------------------------------
def workload(cfg: int, **overrides) -> Workload:
    gl12 = tuple(float(x) for x in gauss_legendre_imag_axis(12))
    gl16 = tuple(float(x) for x in gauss_legendre_imag_axis(16))
    if cfg == 0:
        wl = Workload(name="npb64_nk8_8x32_4w", cfg=0, npb=64, nq=1, nspin=1, nk=8,
                      nocc=8, nunocc=32, omega=(0.1, 0.5, 2.0, 8.0), ztype="c128",
                      unocc_range=(0.05, 3.0), paths=("fp64",))
    elif cfg == 1:
        wl = Workload(name="npb512_nk64_40x300_12w", cfg=1, npb=512, nq=1, nspin=1, nk=64,
                      nocc=40, nunocc=300, omega=gl12, ztype="c128",
                      unocc_range=(0.03, 3.0), paths=("fp64", "fp32"))
    elif cfg == 2:
        wl = Workload(name="npb2048_nk16_200x1200_12w", cfg=2, npb=2048, nq=1, nspin=1, nk=16,
                      nocc=200, nunocc=1200, omega=gl12, ztype="c64",
                      unocc_range=(0.05, 3.0), paths=("bf16x3", "fp64"))
    elif cfg == 3:
        wl = Workload(name="32q_npb384_nk16_ragged_12w", cfg=3, npb=384, nq=32, nspin=1,
                      nk=16, nocc=(16, 64), nunocc=(100, 400), omega=gl12,
                      ztype="c64", unocc_range=(0.05, 3.0), paths=("fp32",))
    elif cfg == 4:
        wl = Workload(name="spin2_metal_npb1024_nk128_16w", cfg=4, npb=1024, nq=1,
                      nspin=2, nk=128, nocc=(52, 68), nunocc=500, omega=gl16,
                      ztype="c64", delta_min=1e-4, occ_range=(-0.8, 0.0),
                      unocc_range=(0.0, 3.0), metallic=True,
                      paths=("bf16x3", "fp64"))
    elif cfg == 5:
        # Exchange self-energy (Eq.(sigx)) at the (InAs)4(GaSb)4 sizes of the
        # paper's system-size table: nqp = 287 quasiparticle states (the Z
        # columns), 92 occupied intermediate states n' (nocc) and 2097
        # product-basis functions mu (nunocc) per k-point, 16 k-points.
        wl = Workload(name="sigx_nqp287_nocc92_npb2097", cfg=5, npb=287, nq=1, nspin=1,
                      nk=16, nocc=92, nunocc=2097, omega=(0.0,), ztype="c128",
                      paths=("fp64", "fp32", "bf16x3"))
    elif cfg == 6:
        # Imaginary-axis correlation self-energy I^c (Eq.(sigci)) at the
        # (InAs)2(GaSb)2 sizes of the paper's system-size table: nqp = 206
        # quasiparticle states, nall = 361 intermediate states n' (92
        # occupied), 1356 product-basis functions mu, 16 k-points; 11
        # imaginary frequencies including w = 0 (0 and 10 Gauss-Legendre
        # nodes mapped to [0, inf)).
        mesh = (0.0,) + tuple(float(x) for x in gauss_legendre_imag_axis(10))
        wl = Workload(name="sigc_nqp206_nall361_npb1356_nk16_11w", cfg=6, npb=206, nq=1,
                      nspin=1, nk=16, nocc=361, nunocc=1356, omega=mesh, ztype="c128",
                      nval=92, paths=("fp64", "bf16x3"))
    else:
        raise ValueError(f"unknown workload {cfg}")
    if overrides:
        wl = wl.replace(**overrides)
    return wl
