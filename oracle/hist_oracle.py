"""CPU oracle of the paper's real-axis route for the polarization (test
infrastructure): the anti-Hermitian part accumulated into histogram bins
(Eq.(impolf), Eq.(tetw)) and the Hilbert transform (Eq.(hilbert)) to any
imaginary or real frequency.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module; it shares no code with the GPU
library.

Reading (the tetrahedron weights of Eq.(tetw) need a k-point mesh, which a
synthetic workload does not have; a uniform spread stands in for them):

* Bins j = [e_j, e_{j+1}) for edges 0 < e_0 < e_1 < ... < e_nb (a first
  edge at 0 would make the bin average of 2x / x^2 at w = 0 diverge).
* A pair (n, n') of a block enters as for chi0: D = eps_unocc[n'] -
  eps_occ[n] > 0 and D >= delta_min.  Its weight w_k is spread uniformly
  over [D (1 - sigma), D (1 + sigma)] (0 <= sigma < 1; sigma = 0 puts all of
  it at D, in the bin with e_j <= D < e_{j+1}); the fraction of that interval
  inside bin j is the pair's bin weight.  Weight outside [e_0, e_nb) is
  dropped.
* S_j = sum_pairs w_j(pair) conj(Z_pair) Z_pair^T (Hermitian, >= 0), and the
  stored histogram is hist_j = -S_j: bin j's integral of the anti-Hermitian
  part of chi0 along the real axis is pi hist_j (Eq.(impolf) with the
  transition energies distributed uniformly within each bin).
* Hilbert transform, with the spectral density uniform within each bin:
  imaginary axis
    chi0(i w) = sum_j c_j(w) hist_j,
    c_j(w) = (1/h_j) int_bin 2x / (x^2 + w^2) dx
           = [ln(e_{j+1}^2 + w^2) - ln(e_j^2 + w^2)] / h_j;
  real axis (w >= 0, not on an edge)
    chi0(w) = sum_j c_j(w) hist_j,
    c_j(w) = [ln|e_{j+1} - w| - ln|e_j - w| + ln(e_{j+1} + w) - ln(e_j + w)] / h_j
             + i pi [w in bin j] / h_j,
  the principal value of (1/h_j) int_bin [1/(x - w) + 1/(x + w)] dx plus the
  density term.  Its Hermitian part is the paper's Re Pi, the other Im Pi.

Pins live in ``tests/pins_hist.py``; none of these functions is "parity
unpinned".
"""
from __future__ import annotations

from fractions import Fraction
from typing import Iterable, List, Sequence, Tuple

import numpy as np

from .chi0_oracle import InvalidPairs, _CompensatedSum, _check_pairs, pair_delta, pair_included


def check_edges(edges: Sequence[float]) -> np.ndarray:
    e = np.asarray(edges, np.float64)
    if e.ndim != 1 or e.size < 2 or not e[0] > 0 or np.any(np.diff(e) <= 0):
        raise ValueError("edges must be strictly increasing, > 0, at least two")
    return e


def bin_fractions(delta: float, edges: Sequence[float], sigma: float) -> List[Tuple[int, float]]:
    """[(j, fraction of the pair's weight in bin j)] for one transition
    energy; fractions outside the edges are dropped."""
    e = check_edges(edges)
    nb = e.size - 1
    if sigma == 0.0:
        if delta < e[0] or delta >= e[-1]:
            return []
        j = int(np.searchsorted(e, delta, side="right")) - 1
        return [(j, 1.0)]
    lo, hi = delta * (1.0 - sigma), delta * (1.0 + sigma)
    width = hi - lo
    out = []
    for j in range(nb):
        a, b = max(lo, e[j]), min(hi, e[j + 1])
        if b > a:
            out.append((j, (b - a) / width))
    return out


def pair_bin_table(eps_occ, eps_unocc, edges, sigma, delta_min, wk) -> np.ndarray:
    """[nb][nocc * nunocc] bin weights w_k * fraction of every pair."""
    e = check_edges(edges)
    d = pair_delta(eps_occ, eps_unocc).reshape(-1)
    inc = pair_included(d, delta_min)
    out = np.zeros((e.size - 1, d.size))
    for p in np.nonzero(inc)[0]:
        for j, f in bin_fractions(float(d[p]), e, sigma):
            out[j, p] = wk * f
    return out


def pair_bins(eps_occ, eps_unocc, edges, sigma, delta_min, wk, nslots: int = 8):
    """The bin weights of every pair in sparse form, vectorised for large
    blocks: (bins [K, nslots] with -1 for unused slots, weights [K, nslots]),
    slot t of a pair holding its t-th bin in increasing order.  The same
    arithmetic as ``bin_fractions`` (pinned equal to ``pair_bin_table``)."""
    e = check_edges(edges)
    nb = e.size - 1
    d = pair_delta(eps_occ, eps_unocc).reshape(-1)
    inc = pair_included(d, delta_min)
    bins = np.full((d.size, nslots), -1, np.int64)
    w = np.zeros((d.size, nslots))
    if sigma == 0.0:
        ok = inc & (d >= e[0]) & (d < e[-1])
        j = np.searchsorted(e, d, side="right") - 1
        bins[ok, 0] = j[ok]
        w[ok, 0] = wk * 1.0
        return bins, w
    lo, hi = d * (1.0 - sigma), d * (1.0 + sigma)
    width = hi - lo
    j0 = np.maximum(np.searchsorted(e, lo, side="right") - 1, 0)
    t = np.zeros(d.size, np.int64)
    for k in range(nslots + 1):
        j = j0 + k
        live = inc & (j < nb)
        jj = np.minimum(j, nb - 1)
        live &= e[jj] < hi
        a = np.maximum(lo, e[jj])
        b = np.minimum(hi, e[jj + 1])
        take = live & (b > a)
        if np.any(take & (t >= nslots)):
            raise ValueError("more bins per pair than slots")
        idx = np.nonzero(take)[0]
        bins[idx, t[idx]] = jj[idx]
        w[idx, t[idx]] = wk * ((b[idx] - a[idx]) / width[idx])
        t[idx] += 1
    return bins, w


def hist_block(z: np.ndarray, eps_occ, eps_unocc, wk, edges, sigma, delta_min) -> np.ndarray:
    """hist_j = -S_j of one block, [nb][npb][npb]."""
    z = np.asarray(z, np.complex128)
    nocc, nunocc, npb = z.shape
    a = z.reshape(nocc * nunocc, npb)
    t = pair_bin_table(eps_occ, eps_unocc, edges, sigma, delta_min, wk)
    out = np.zeros((t.shape[0], npb, npb), np.complex128)
    for j in range(t.shape[0]):
        rows = np.nonzero(t[j])[0]
        if rows.size:
            ar = a[rows]
            out[j] = -(ar.conj().T @ (t[j, rows][:, None] * ar))
    return out


def hist_ref(blocks: Iterable, npb: int, edges, sigma: float, delta_min: float = 0.0,
             strict: bool = True) -> np.ndarray:
    """hist_j summed over blocks (compensated), [nb][npb][npb].  Pairs with
    D <= 0 are rejected (InvalidPairs) unless strict=False skips them."""
    e = check_edges(edges)
    acc = _CompensatedSum((e.size - 1, npb, npb))
    for z, eo, eu, wk in blocks:
        _check_pairs(eo, eu, strict)
        acc.add(hist_block(z, eo, eu, wk, e, sigma, delta_min))
    return acc.value()


def hist_brute(blocks: Iterable, npb: int, edges, sigma: float, delta_min: float = 0.0,
               strict: bool = True) -> np.ndarray:
    """Explicit loops over pairs, bins and (I, J) (tiny inputs only)."""
    e = check_edges(edges)
    out = np.zeros((e.size - 1, npb, npb), np.complex128)
    for z, eo, eu, wk in blocks:
        _check_pairs(eo, eu, strict)
        for n in range(len(eo)):
            for m in range(len(eu)):
                d = float(eu[m] - eo[n])
                if not (d > 0 and d >= delta_min):
                    continue
                for j, f in bin_fractions(d, e, sigma):
                    for i in range(npb):
                        for k in range(npb):
                            out[j, i, k] -= wk * f * np.conj(z[n, m, i]) * z[n, m, k]
    return out


def hist_exact(blocks, npb: int, edges: Sequence[Fraction], delta_min=Fraction(0),
               strict: bool = True):
    """Exact histogram for sigma = 0 with rational energies, weights and
    (re, im) Fraction Z entries: [nb][npb][npb] of (re, im)."""
    nb = len(edges) - 1
    out = [[[(Fraction(0), Fraction(0)) for _ in range(npb)] for _ in range(npb)] for _ in range(nb)]
    for z, eo, eu, wk in blocks:
        if strict and any(not (u - o > 0) for o in eo for u in eu):
            raise InvalidPairs("pair(s) with D <= 0")
        for n in range(len(eo)):
            for m in range(len(eu)):
                d = eu[m] - eo[n]
                if not (d > 0 and d >= delta_min):
                    continue
                js = [j for j in range(nb) if edges[j] <= d < edges[j + 1]]
                for j in js:
                    for i in range(npb):
                        ar, ai = z[n][m][i]
                        for k in range(npb):
                            br, bi = z[n][m][k]
                            re = ar * br + ai * bi
                            im = ar * bi - ai * br
                            r0, i0 = out[j][i][k]
                            out[j][i][k] = (r0 - wk * re, i0 - wk * im)
    return out


def hist_entries(block_columns, edges, sigma: float, entries: Sequence[Tuple[int, int]],
                 col_index: dict, delta_min: float = 0.0, strict: bool = True) -> np.ndarray:
    """hist_j[I][J] of the listed entries only, [nb][len(entries)].
    ``block_columns`` yields (Zc[K, ncols], eps_occ, eps_unocc, w_k) with Zc
    holding the columns of Z (pairs n-major) listed in ``col_index``."""
    e = check_edges(edges)
    nb = e.size - 1
    ii = np.array([col_index[i] for i, _ in entries])
    jj = np.array([col_index[j] for _, j in entries])
    acc = _CompensatedSum((nb, len(entries)))
    for zc, eo, eu, wk in block_columns:
        _check_pairs(eo, eu, strict)
        zc = np.asarray(zc, np.complex128)
        bins, w = pair_bins(eo, eu, e, sigma, delta_min, wk)
        prod = zc[:, ii].conj() * zc[:, jj]                    # [K, entries]
        used = bins >= 0
        b = bins[used]
        part = np.zeros((nb, len(entries)), np.complex128)
        for k in range(len(entries)):
            v = (w * prod[:, k][:, None])[used]
            part[:, k] = -(np.bincount(b, weights=v.real, minlength=nb)
                           + 1j * np.bincount(b, weights=v.imag, minlength=nb))
        acc.add(part)
    return acc.value()


def hilbert_imag(edges, omega: Sequence[float]) -> np.ndarray:
    """c_j(i w) of every (w, bin), float64 [nomega][nb].  The difference of
    logarithms is evaluated as log1p((e_{j+1} - e_j)(e_{j+1} + e_j) /
    (e_j^2 + w^2)), which keeps full relative accuracy when w is far above
    the bin (the plain difference cancels there)."""
    e = check_edges(edges)
    w = np.asarray(omega, np.float64)[:, None]
    lo, hi = e[None, :-1], e[None, 1:]
    h = hi - lo
    return np.log1p(h * (hi + lo) / (lo * lo + w * w)) / h


def hilbert_real(edges, omega: Sequence[float]) -> np.ndarray:
    """c_j(w) of every real (w, bin), complex128 [nreal][nb]; w must not be an
    edge.  ln|e_{j+1} - w| - ln|e_j - w| is log1p(h / (e_j - w)) for w
    outside the bin and the plain difference inside it; ln(e_{j+1} + w) -
    ln(e_j + w) is log1p(h / (e_j + w))."""
    e = check_edges(edges)
    om = np.asarray(omega, np.float64)
    if np.any(np.isin(om, e)):
        raise ValueError("a real frequency lies on a bin edge")
    w = om[:, None]
    lo, hi = e[None, :-1], e[None, 1:]
    h = hi - lo
    inside = (w > lo) & (w < hi)
    with np.errstate(divide="ignore", invalid="ignore"):
        near = np.where(inside, np.log(np.abs(hi - w)) - np.log(np.abs(lo - w)),
                        np.log1p(h / (lo - w)))
        far = np.log1p(h / (lo + w))
    return (near + far) / h + 1j * np.pi * inside / h


def hilbert_apply(coeff: np.ndarray, hist: np.ndarray) -> np.ndarray:
    """chi0_i = sum_j coeff[i][j] hist_j, [nout][npb][npb]."""
    return np.tensordot(np.asarray(coeff), hist, axes=([1], [0]))


def hist_workload_blocks(wl, q: int = 0):
    """Stream (Z, eps_occ, eps_unocc, w_k) of a synthetic workload."""
    for blk in wl.blocks(q):
        eo, eu = wl.energies(blk)
        yield wl.z_block(blk).astype(np.complex128), eo, eu, blk.wk


def log_edges(e0: float, ratio: float, emax: float) -> np.ndarray:
    """Logarithmic bin edges e0 * ratio^j up to the first edge above emax
    (the paper's histogram mesh is 1e-5 * 1.03^j Ry)."""
    n = int(np.ceil(np.log(emax / e0) / np.log(ratio))) + 1
    return e0 * ratio ** np.arange(n + 1)
