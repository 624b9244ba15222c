"""Pins of the histogram + Hilbert oracle (oracle/hist_oracle.py) against
what Eq.(impolf), Eq.(hilbert), the reading of the bin weights and the
mathematics fix: hand-computed dyadic bin fractions, exact rational
histograms, explicit loops, the bin average of the direct transition weight
by adaptive quadrature (imaginary axis) and by principal-value quadrature
(real axis), convergence to the direct chi0 of Eq.(polfx) as the bins
shrink, Kramers-Kronig consistency at w = 0, the density term and its sum
rule, and the sign / order properties of the result."""
import math
import warnings
from fractions import Fraction

import numpy as np

import oracle.chi0_oracle as direct


def _close(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def pin_fractions_hand(orc):
    """D = 1, sigma = 1/4: the spread covers [3/4, 5/4]; with edges
    {1/2, 7/8, 3/2} bin 0 holds 1/8 of its width 1/2 (= 1/4) and bin 1 the
    remaining 3/4.  sigma = 0: the bin whose left edge is D, ties included;
    D at or beyond the last edge, or below the first, is dropped."""
    fails = []
    got = orc.bin_fractions(1.0, [0.5, 0.875, 1.5], 0.25)
    if got != [(0, 0.25), (1, 0.75)]:
        fails.append(f"dyadic fractions {got}")
    if orc.bin_fractions(0.875, [0.5, 0.875, 1.5], 0.0) != [(1, 1.0)]:
        fails.append("tie at an edge not in the right-hand bin")
    if orc.bin_fractions(1.5, [0.5, 0.875, 1.5], 0.0) != []:
        fails.append("last edge not excluded")
    if orc.bin_fractions(0.25, [0.5, 0.875, 1.5], 0.0) != []:
        fails.append("below the first edge not dropped")
    got = orc.bin_fractions(1.0, [0.9, 1.1, 2.0], 0.5)       # [0.5, 1.5]: part dropped
    if not _close([f for _, f in got], [0.2, 0.4], 1e-15) or [j for j, _ in got] != [0, 1]:
        fails.append(f"partly outside: {got}")
    return fails


def pin_exact_and_brute(orc):
    """sigma = 0, dyadic energies, small-integer Z: exact rational histogram
    = explicit loops = reference; a delta_min tie is included."""
    fails = []
    rng = np.random.default_rng(4)
    npb = 3
    edges = [Fraction(1, 8), Fraction(1, 2), Fraction(1), Fraction(5, 2)]
    blocks, ex_in = [], []
    for nocc, nunocc, wk in ((2, 3, Fraction(1, 2)), (3, 2, Fraction(1, 4))):
        zr = rng.integers(-3, 4, (nocc, nunocc, npb))
        zi = rng.integers(-3, 4, (nocc, nunocc, npb))
        eo = [Fraction(-int(x), 16) for x in rng.integers(0, 8, nocc)]
        eu = [Fraction(int(x), 8) for x in rng.integers(1, 16, nunocc)]
        blocks.append((zr + 1j * zi, np.array([float(x) for x in eo]),
                       np.array([float(x) for x in eu]), float(wk)))
        ex_in.append(([[[(Fraction(int(zr[a, b, c])), Fraction(int(zi[a, b, c])))
                         for c in range(npb)] for b in range(nunocc)] for a in range(nocc)],
                      eo, eu, wk))
    fe = [float(x) for x in edges]
    ex = orc.hist_exact(ex_in, npb, edges, Fraction(1, 4))
    ex = np.array([[[float(r) + 1j * float(i) for r, i in row] for row in m] for m in ex])
    ref = orc.hist_ref(blocks, npb, fe, 0.0, 0.25)
    if not _close(ref, ex, 1e-15):
        fails.append("reference != exact")
    if not _close(orc.hist_brute(blocks, npb, fe, 0.0, 0.25), ex, 1e-15):
        fails.append("loops != exact")
    if not _close(orc.hist_brute(blocks, npb, fe, 0.3, 0.0), orc.hist_ref(blocks, npb, fe, 0.3, 0.0), 1e-14):
        fails.append("loops != reference with spread")
    ent = [(0, 2), (1, 1), (2, 0)]
    cols = [(z.reshape(-1, npb), eo, eu, wk) for z, eo, eu, wk in blocks]
    got = orc.hist_entries(cols, fe, 0.3, ent, {0: 0, 1: 1, 2: 2})
    full = orc.hist_ref(blocks, npb, fe, 0.3, 0.0)
    if not _close(got, np.array([[full[j, a, b] for a, b in ent] for j in range(full.shape[0])]), 1e-14):
        fails.append("entry sampler != reference")
    return fails


def pin_single_pair_imag(orc):
    """One pair, D in bin [L, R] (sigma = 0): chi0(i w) from the histogram is
    the direct Eq.(polfx) weight -2 w_k x / (x^2 + w^2) averaged over x in the
    bin (adaptive quadrature) times conj(z) z^T."""
    from scipy.integrate import quad
    fails = []
    z = np.array([[[1 + 2j, -0.5j, 0.25]]])
    eo, eu, wk = np.array([-0.3]), np.array([0.4]), 0.5       # D = 0.7
    edges = [0.1, 0.55, 0.9, 2.0]
    hist = orc.hist_ref([(z, eo, eu, wk)], 3, edges, 0.0)
    omegas = [0.0, 0.05, 0.8, 7.0]
    got = orc.hilbert_apply(orc.hilbert_imag(edges, omegas), hist)
    zz = np.conj(z[0, 0])[:, None] * z[0, 0][None, :]
    for k, w in enumerate(omegas):
        avg = quad(lambda x: -2 * wk * x / (x * x + w * w), 0.55, 0.9, epsabs=0, epsrel=1e-13)[0] / 0.35
        if not _close(got[k], avg * zz, 1e-13):
            fails.append(f"single pair, w = {w}")
    return fails


def pin_single_pair_real(orc):
    """One pair, real axis: the Hermitian part is the principal value of the
    real-axis weight 1/(w - x) - 1/(w + x) averaged over the bin (scipy's
    Cauchy-weight quadrature) and the anti-Hermitian part -pi w_k / h for w
    inside the bin, 0 outside."""
    from scipy.integrate import quad
    fails = []
    z = np.array([[[1.0 + 0.5j, 2.0 - 1j]]])
    eo, eu, wk = np.array([-0.2]), np.array([0.5]), 0.25      # D = 0.7
    edges = [0.1, 0.55, 0.9, 2.0]
    hist = orc.hist_ref([(z, eo, eu, wk)], 2, edges, 0.0)
    omegas = [0.0, 0.3, 0.7, 1.4]
    got = orc.hilbert_apply(orc.hilbert_real(edges, omegas), hist)
    zz = np.conj(z[0, 0])[:, None] * z[0, 0][None, :]
    for k, w in enumerate(omegas):
        with warnings.catch_warnings():
            warnings.simplefilter("ignore")
            if 0.55 < w < 0.9:      # 1/(w - x) = -1/(x - w): Cauchy weight at x = w
                pv = -quad(lambda x: 1.0, 0.55, 0.9, weight="cauchy", wvar=w)[0]
            else:
                pv = quad(lambda x: 1.0 / (w - x), 0.55, 0.9, epsabs=0, epsrel=1e-13)[0]
            pv -= quad(lambda x: 1.0 / (w + x), 0.55, 0.9, epsabs=0, epsrel=1e-13)[0]
        herm = wk * pv / 0.35
        anti = -math.pi * wk / 0.35 if 0.55 < w < 0.9 else 0.0
        if not _close(got[k], (herm + 1j * anti) * zz, 1e-11):
            fails.append(f"real axis single pair, w = {w}")
    return fails


def pin_converges_to_direct(orc):
    """Log bins of ratio r and sigma = 0: chi0(i w) from the histogram tends
    to the direct chi0 of Eq.(polfx).  Each pair's weight f(D) = 2D/(D^2+w^2)
    is replaced by its average over D's bin, and |f'/f| <= 1/x, so the
    relative error per pair is at most r (r - 1): first order in the bin
    width (the spread's centre is the bin's, not D); it must fall by about 2
    when ln r halves."""
    fails = []
    rng = np.random.default_rng(9)
    npb = 6
    blocks = []
    for _ in range(2):
        z = rng.standard_normal((3, 5, npb)) + 1j * rng.standard_normal((3, 5, npb))
        blocks.append((z, np.sort(rng.uniform(-0.8, 0, 3)), np.sort(rng.uniform(0.05, 3, 5)), 0.5))
    omegas = [0.0, 0.1, 1.0, 5.0]
    ref = direct.chi0_ref(blocks, npb, omegas)
    errs = []
    for r in (1.02, 1.01):
        edges = orc.log_edges(0.01, r, 4.0)
        hist = orc.hist_ref(blocks, npb, edges, 0.0)
        got = orc.hilbert_apply(orc.hilbert_imag(edges, omegas), hist)
        e = max(_rel(got[k], ref[k]) for k in range(len(omegas)))
        if e > r * (r - 1):
            fails.append(f"ratio {r}: error {e} above bound")
        errs.append(e)
    if not (1.5 < errs[0] / errs[1] < 3):
        fails.append(f"no first-order convergence {errs}")
    return fails


def pin_real_imag_consistency(orc):
    """Kramers-Kronig: the real-axis Hermitian part at w = 0 equals the
    imaginary-axis value at w = 0; the density term integrates to pi times
    the total histogram (sum rule); sigma > 0 spreads but keeps the total
    weight of a pair whose spread lies inside the edges."""
    fails = []
    rng = np.random.default_rng(12)
    npb = 4
    z = rng.standard_normal((2, 3, npb)) + 1j * rng.standard_normal((2, 3, npb))
    blk = [(z, np.array([-0.4, -0.1]), np.array([0.2, 0.9, 1.7]), 0.5)]
    edges = orc.log_edges(0.05, 1.1, 3.0)
    for sigma in (0.0, 0.07):
        hist = orc.hist_ref(blk, npb, edges, sigma)
        a = orc.hilbert_apply(orc.hilbert_imag(edges, [0.0]), hist)[0]
        b = orc.hilbert_apply(orc.hilbert_real(edges, [0.0]), hist)[0]
        if not _close(a, b, 1e-14):
            fails.append(f"w = 0 mismatch, sigma {sigma}")
        centres = 0.5 * (edges[:-1] + edges[1:])
        dens = orc.hilbert_apply(np.imag(orc.hilbert_real(edges, centres)), hist)
        integral = np.tensordot(np.diff(edges), dens, axes=(0, 0))
        if not _close(integral, math.pi * hist.sum(axis=0), 1e-13):
            fails.append(f"density sum rule, sigma {sigma}")
        total = hist.sum(axis=0)
        zz = sum(0.5 * np.conj(z[n, m])[:, None] * z[n, m][None, :] for n in range(2) for m in range(3))
        if not _close(total, -zz, 1e-14):
            fails.append(f"total weight not w_k per pair, sigma {sigma}")
    return fails


def pin_order_properties(orc):
    """hist_j <= 0 (Hermitian, negative semidefinite); chi0(i w) Hermitian,
    <= 0 and increasing in w (Loewner); the real-axis anti-Hermitian part
    <= 0."""
    fails = []
    rng = np.random.default_rng(2)
    npb = 5
    blocks = [(rng.standard_normal((3, 4, npb)) + 1j * rng.standard_normal((3, 4, npb)),
               np.sort(rng.uniform(-0.8, 0, 3)), np.sort(rng.uniform(0.05, 3, 4)), 0.25)]
    edges = orc.log_edges(0.02, 1.07, 4.0)
    hist = orc.hist_ref(blocks, npb, edges, 0.04)
    for j in range(hist.shape[0]):
        if not _close(hist[j], hist[j].conj().T, 1e-15) or np.linalg.eigvalsh(hist[j]).max() > 1e-13:
            fails.append(f"bin {j} not Hermitian <= 0")
            break
    w = [0.0, 0.3, 1.0, 4.0]
    c = orc.hilbert_apply(orc.hilbert_imag(edges, w), hist)
    for k in range(len(w)):
        if np.linalg.eigvalsh(c[k]).max() > 1e-12:
            fails.append(f"chi0(i w) not <= 0 at {w[k]}")
        if k and np.linalg.eigvalsh(c[k] - c[k - 1]).min() < -1e-12:
            fails.append(f"not increasing at {w[k]}")
    wr = [0.33, 1.21]
    r = orc.hilbert_apply(orc.hilbert_real(edges, wr), hist)
    for k in range(2):
        anti = (r[k] - r[k].conj().T) / 2j
        if np.linalg.eigvalsh(anti).max() > 1e-12:
            fails.append("real-axis anti-Hermitian part not <= 0")
    return fails


def pin_delta_min_as_direct(orc):
    """The pair filter is the chi0 one: a pair below delta_min contributes
    nothing, a tie is included, and a pair with D <= 0 is rejected (or,
    when asked for, skipped)."""
    fails = []
    z = np.ones((1, 3, 2), complex)
    eo = np.array([0.0])
    eu = np.array([-0.1, 0.25, 0.5])                # D = -0.1, 0.25, 0.5
    edges = [0.01, 1.0]
    h = orc.hist_ref([(z, eo, eu, 1.0)], 2, edges, 0.0, 0.25, strict=False)
    if not _close(h[0], -2 * np.ones((2, 2)), 1e-15):
        fails.append("delta_min filter")
    try:
        orc.hist_ref([(z, eo, eu, 1.0)], 2, edges, 0.0, 0.25)
        fails.append("a pair with D <= 0 was accepted")
    except ValueError:
        pass
    return fails


def pin_sparse_table(orc):
    """The vectorised sparse bin table equals the per-pair definition
    exactly (same arithmetic), with and without spread, for random energies
    around random log meshes, ties at edges included."""
    fails = []
    rng = np.random.default_rng(17)
    for sigma in (0.0, 0.015, 0.2):
        edges = orc.log_edges(0.05, 1.03 if sigma < 0.1 else 1.2, 3.5)
        eo = np.sort(rng.uniform(-0.8, 0, 7))
        eu = np.concatenate([np.sort(rng.uniform(0.05, 3.0, 40)), edges[[5, 9]] + eo[0]])
        dense = orc.pair_bin_table(eo, eu, edges, sigma, 0.1, 0.25)
        bins, w = orc.pair_bins(eo, eu, edges, sigma, 0.1, 0.25)
        rebuilt = np.zeros_like(dense)
        for p in range(bins.shape[0]):
            for t in range(bins.shape[1]):
                if bins[p, t] >= 0:
                    rebuilt[bins[p, t], p] += w[p, t]
        if not np.array_equal(rebuilt, dense):
            fails.append(f"sparse table != definition at sigma {sigma}")
    return fails


PINS = [pin_sparse_table, pin_fractions_hand, pin_exact_and_brute, pin_single_pair_imag, pin_single_pair_real,
        pin_converges_to_direct, pin_real_imag_consistency, pin_order_properties,
        pin_delta_min_as_direct]


def run_all(orc):
    return {p.__name__: p(orc) for p in PINS}
