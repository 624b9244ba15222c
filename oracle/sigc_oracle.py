"""CPU oracle for the imaginary-axis part I^c of the correlation self-energy
(test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module; it shares no code with the GPU
library.

Eq.(sigci), discretised: for the quasiparticle states n, m of one q-point,
  I^c[n][m] = - sum_k w_k sum_{n'} sum_i w^I_i(eps_qn - eps_{q-k,n'})
              sum_{mu, nu} conj(Z_k[n'][mu][n]) W^c_k(i w_i)[mu][nu] Z_k[n'][nu][m]
with Z_k[n'][mu][n] the product-basis matrix element of Eq.(defz) between the
function mu of k and the states (q-k, n'), (q, n); n' runs over all
intermediate states (occupied and unoccupied); W^c_k(i w_i) = sqrt(v) (eps^-1
- 1) sqrt(v) of Eq.(wc) on the imaginary-frequency mesh {w_i}; w_k a per-k
weight (1 for the bare Brillouin-zone sum as printed).  The row index n alone
sets the energy denominator, so I^c is not Hermitian in general.

The integration weights w^I_i(dE) (Section "Self-energy", Aryasetiawan-
Gunnarsson method, cited but not printed) are read as follows.  W^c is even
in w along the imaginary axis, so
  int dw/(2 pi) X(iw) / (dE - iw) = (1/pi) int_0^inf X(iw) dE / (dE^2 + w^2) dw,
the odd part of the integrand cancelling.  X is replaced by its interpolant on
the mesh 0 <= w_0 < w_1 < ... < w_{n-1}: constant X(w_0) on [0, w_0],
piecewise linear between nodes, and X(w_{n-1}) (w_{n-1}/w)^2 beyond the last
node (W^c decays as 1/w^2 there, since chi0 does).  The Lorentzian factor is
integrated exactly against each node's basis function; w^I_i(dE) is that
integral.  At dE = 0 exactly the weights are 0 (the principal value; the
integrand 1/(-iw) is odd).  The weights are odd in dE and have no units.

The weights are evaluated with mpmath at 40+ significant digits from the
plain primitives atan(w/dE) and (dE/2) ln(dE^2 + w^2), so cancellation
between them cannot reach the double-precision result; the contraction
follows the order of the paper's self-energy algorithm (weighted Z, then
Z_w^H W^c summed over the mesh, then the product with Z).

Pins live in ``tests/pins_sigc.py``; none of these functions is "parity
unpinned".
"""
from __future__ import annotations

import math
from fractions import Fraction
from typing import Iterable, Sequence, Tuple

import mpmath
import numpy as np

from .chi0_oracle import _CompensatedSum

SigcBlock = Tuple[np.ndarray, np.ndarray, np.ndarray, float]
# (Z[nall, npb, nqp] complex, W^c[nomega, npb, npb] complex, eps_mid[nall], w_k)


def ag_weights(delta: float, mesh: Sequence[float]) -> np.ndarray:
    """w^I_i(dE) for i over the mesh, float64 (rounded from >= 40 digits)."""
    mesh = [float(x) for x in mesh]
    n = len(mesh)
    if n == 0:
        return np.zeros(0)
    if any(mesh[i + 1] <= mesh[i] for i in range(n - 1)) or mesh[0] < 0:
        raise ValueError("mesh must be strictly increasing and >= 0")
    if delta == 0.0:
        return np.zeros(n)
    # digits lost to cancellation grow like 2 log10(mesh scale / |dE|) at
    # small |dE| (the tail term) and like 2 log10(|dE| / mesh step) at large
    # |dE| (differences of nearly equal primitives): add them to the working
    # precision
    scale = max(abs(mesh[-1]), 1e-300)
    lo = min(mesh[i + 1] - mesh[i] for i in range(n - 1)) if n > 1 else scale
    ls, ld, ll = math.log10(scale), math.log10(abs(delta)), math.log10(lo)
    extra = 2 * max(0.0, ls - ld) + 2 * max(0.0, ld - ll) + max(0.0, ls - ll)
    with mpmath.workdps(40 + int(extra) + 5):
        d = mpmath.mpf(delta)
        om = [mpmath.mpf(x) for x in mesh]
        pi = mpmath.pi

        def f0(w):                       # primitive of dE / (dE^2 + w^2)
            return mpmath.atan(w / d)

        def f1(w):                       # primitive of w dE / (dE^2 + w^2)
            return d / 2 * mpmath.log(d * d + w * w)

        w = [mpmath.mpf(0)] * n
        # [0, w_0]: constant extension of the first node
        w[0] += f0(om[0]) - f0(mpmath.mpf(0))
        # interior intervals: hat functions
        for j in range(n - 1):
            a, b = om[j], om[j + 1]
            h = b - a
            i0 = f0(b) - f0(a)
            i1 = f1(b) - f1(a)
            w[j] += (b * i0 - i1) / h          # (b - w) / h on [a, b]
            w[j + 1] += (i1 - a * i0) / h      # (w - a) / h on [a, b]
        # tail: X(w_{n-1}) (c / w)^2 on [c, inf);
        # int_c^inf c^2 dE / (w^2 (dE^2 + w^2)) dw
        #   = (c^2 / dE) [1/c - (1/|dE|)(pi/2 - atan(c/|dE|))]
        c = om[-1]
        if c > 0:
            ad = abs(d)
            w[n - 1] += c * c / d * (1 / c - (pi / 2 - mpmath.atan(c / ad)) / ad)
        else:                                  # one node at w = 0: constant X
            w[n - 1] += (pi / 2) * mpmath.sign(d)
        return np.array([float(x / pi) for x in w])


def ag_weight_table(eps_qp: np.ndarray, eps_mid: np.ndarray,
                    mesh: Sequence[float]) -> np.ndarray:
    """[nall][nqp][nomega]: w^I_i(eps_qp[n] - eps_mid[n'])."""
    eps_qp = np.asarray(eps_qp, np.float64)
    eps_mid = np.asarray(eps_mid, np.float64)
    out = np.empty((len(eps_mid), len(eps_qp), len(mesh)))
    cache = {}
    for a, e1 in enumerate(eps_mid):
        for n, e0 in enumerate(eps_qp):
            d = float(e0 - e1)
            if d not in cache:
                cache[d] = ag_weights(d, mesh)
            out[a, n] = cache[d]
    return out


def sigc_block(z: np.ndarray, wc: np.ndarray, weights: np.ndarray,
               wk: float) -> np.ndarray:
    """Contribution of one k-point, [nqp, nqp], given its weight table
    weights[n'][n][i]: for each n', Z_w = Z w_i (per column n), then
    ZW = sum_i Z_w^H W^c_i, then -w_k ZW Z."""
    z = np.asarray(z, np.complex128)
    wc = np.asarray(wc, np.complex128)
    nall, npb, nqp = z.shape
    out = np.zeros((nqp, nqp), np.complex128)
    for a in range(nall):
        za = z[a]                                   # [mu, n]
        zw_w = np.zeros((nqp, npb), np.complex128)  # ZW[n, nu]
        for i in range(wc.shape[0]):
            zwi = za * weights[a, :, i][None, :]
            zw_w += zwi.conj().T @ wc[i]
        out += zw_w @ za
    return -float(wk) * out


def sigc_ref(blocks: Iterable[SigcBlock], eps_qp: np.ndarray,
             mesh: Sequence[float]) -> np.ndarray:
    """I^c[nqp, nqp] summed over k-points with compensated addition."""
    nqp = len(eps_qp)
    acc = _CompensatedSum((nqp, nqp))
    for z, wc, eps_mid, wk in blocks:
        acc.add(sigc_block(z, wc, ag_weight_table(eps_qp, eps_mid, mesh), wk))
    return acc.value()


def sigc_rows(blocks: Iterable[SigcBlock], eps_qp: np.ndarray,
              mesh: Sequence[float], rows: Sequence[int]) -> np.ndarray:
    """Selected rows n of I^c (for sampled checks of large problems):
    out[r][m] = I^c[rows[r]][m]."""
    eps_qp = np.asarray(eps_qp, np.float64)
    rows = list(rows)
    nqp = len(eps_qp)
    acc = _CompensatedSum((len(rows), nqp))
    for z, wc, eps_mid, wk in blocks:
        z = np.asarray(z, np.complex128)
        wc = np.asarray(wc, np.complex128)
        wt = ag_weight_table(eps_qp[rows], eps_mid, mesh)      # [nall][r][i]
        part = np.zeros((len(rows), nqp), np.complex128)
        for a in range(z.shape[0]):
            zr = z[a][:, rows]                                  # [mu, r]
            zw = np.zeros((len(rows), z.shape[1]), np.complex128)
            for i in range(wc.shape[0]):
                zw += (zr * wt[a, :, i][None, :]).conj().T @ wc[i]
            part += zw @ z[a]
        acc.add(-float(wk) * part)
    return acc.value()


def sigc_entries(blocks, eps_qp: np.ndarray, mesh: Sequence[float],
                 entries: Sequence[Tuple[int, int]]) -> np.ndarray:
    """Selected entries I^c[n][m] of a large problem.  ``blocks`` yields
    (zc, cols, W^c, eps_mid, w_k) with zc[n'][mu][j] = Z[n'][mu][cols[j]]
    holding at least the columns n and m of every entry."""
    eps_qp = np.asarray(eps_qp, np.float64)
    rows = sorted({int(n) for n, _ in entries})
    acc = _CompensatedSum((len(entries),))
    for zc, cols, wc, eps_mid, wk in blocks:
        zc = np.asarray(zc, np.complex128)                         # [n', mu, j]
        wc = np.asarray(wc, np.complex128)
        where = {int(c): j for j, c in enumerate(cols)}
        wt = ag_weight_table(eps_qp[rows], eps_mid, mesh)          # [n', row, i]
        wrow = {n: k for k, n in enumerate(rows)}
        part = np.zeros(len(entries), np.complex128)
        for i in range(wc.shape[0]):
            t = np.matmul(wc[i][None, :, :], zc)                   # W_i Z[n'], [n', nu, j]
            s = np.matmul(np.conj(np.transpose(zc, (0, 2, 1))), t)  # [n', j, k]
            for e, (n, m) in enumerate(entries):
                part[e] += np.sum(wt[:, wrow[n], i] * s[:, where[n], where[m]])
        acc.add(-float(wk) * part)
    return acc.value()


def sigc_brute(blocks: Iterable[SigcBlock], eps_qp: np.ndarray,
               mesh: Sequence[float]) -> np.ndarray:
    """Explicit loops over k, n', i, mu, nu, n, m (tiny inputs only)."""
    nqp = len(eps_qp)
    out = np.zeros((nqp, nqp), np.complex128)
    for z, wc, eps_mid, wk in blocks:
        nall, npb, _ = z.shape
        for a in range(nall):
            for n in range(nqp):
                wt = ag_weights(float(eps_qp[n] - eps_mid[a]), mesh)
                for m in range(nqp):
                    s = 0j
                    for i in range(len(mesh)):
                        for mu in range(npb):
                            for nu in range(npb):
                                s += wt[i] * np.conj(z[a, mu, n]) * wc[i, mu, nu] * z[a, nu, m]
                    out[n, m] -= wk * s
    return out


def sigc_contract_exact(blocks, nqp: int):
    """Exact rational contraction with given rational weights: each block is
    (Z[n'][mu][n] as (re, im) Fraction pairs, W[i][mu][nu] likewise,
    weights[n'][n][i] Fractions, w_k Fraction).  Returns [nqp][nqp] (re, im)."""
    out = [[(Fraction(0), Fraction(0)) for _ in range(nqp)] for _ in range(nqp)]

    def mul(x, y):
        return (x[0] * y[0] - x[1] * y[1], x[0] * y[1] + x[1] * y[0])

    for z, wc, wt, wk in blocks:
        nall, npb, nom = len(z), len(z[0]), len(wc)
        for a in range(nall):
            for n in range(nqp):
                for m in range(nqp):
                    sr, si = Fraction(0), Fraction(0)
                    for i in range(nom):
                        for mu in range(npb):
                            zc = (z[a][mu][n][0], -z[a][mu][n][1])
                            for nu in range(npb):
                                p = mul(mul(zc, wc[i][mu][nu]), z[a][nu][m])
                                sr += wt[a][n][i] * p[0]
                                si += wt[a][n][i] * p[1]
                    r0, i0 = out[n][m]
                    out[n][m] = (r0 - wk * sr, i0 - wk * si)
    return out


def sigc_contract(blocks, nqp: int) -> np.ndarray:
    """The contraction of ``sigc_block`` with caller-given weight tables:
    blocks of (Z, W^c, weights[n'][n][i], w_k)."""
    acc = _CompensatedSum((nqp, nqp))
    for z, wc, wt, wk in blocks:
        acc.add(sigc_block(z, wc, np.asarray(wt, np.float64), wk))
    return acc.value()


def sigc_workload_blocks(wl, q: int = 0):
    """Stream (Z, W^c, eps_mid, w_k) of a synthetic correlation workload."""
    for blk in wl.blocks(q):
        yield wl.z_block(blk), wl.wc_block(blk), wl.eps_mid(blk), blk.wk
