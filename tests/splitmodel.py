"""Numpy model of the reduced-precision contractions, used to tell kernel
mistakes apart from the rounding the precision choice itself implies.

The model rounds exactly where the GPU paths round (FP32 weight, FP32 scaled
operand, bf16 round-to-nearest-even hi / lo split) and then sums the products
in FP64, so it differs from the GPU only by the FP32 accumulation of runs.
Test infrastructure; not the oracle.
"""
import numpy as np

import oracle


def bf16_rne(x32):
    """Round float32 values to bfloat16 (nearest, ties to even), as float32."""
    b = np.asarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    r = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return r.astype(np.uint32).view(np.float32)


def split(x32):
    hi = bf16_rne(x32)
    lo = bf16_rne((x32 - hi).astype(np.float32))
    return hi.astype(np.float64), lo.astype(np.float64)


def mirror_lower(m):
    """The GPU computes the lower triangle (row index on the unscaled,
    conjugated side) and mirrors it with conjugation, imaginary diagonal 0;
    the model returns the same Hermitian matrix from its lower triangle
    (its upper triangle has the two sides' roundings swapped)."""
    m = np.asarray(m)
    lo = np.tril(m)
    out = lo + np.conj(np.swapaxes(np.tril(lo, -1), -1, -2))
    d = np.einsum("...ii->...i", out)
    d.imag[...] = 0.0
    return out


def weighted_model(rows, weights, path="bf16x3", lolo=False):
    """-sum_r w_r conj(Z_r)^T Z_r with the GPU's rounding (FP32 weight on the
    Q side, bf16 split), summed in FP64.  rows: complex64 [K, n]."""
    a = np.asarray(rows, np.complex64)
    c32 = np.asarray(weights, np.float64).astype(np.float32)[:, None]
    br = (a.real.astype(np.float32) * c32).astype(np.float32)
    bi = (a.imag.astype(np.float32) * c32).astype(np.float32)
    ar = a.real.astype(np.float32)
    ai = a.imag.astype(np.float32)
    if path == "fp32":
        ar64, ai64, br64, bi64 = (x.astype(np.float64) for x in (ar, ai, br, bi))
        sr = ar64.T @ br64 + ai64.T @ bi64
        si = ar64.T @ bi64 - ai64.T @ br64
    else:
        (arh, arl), (aih, ail) = split(ar), split(ai)
        (brh, brl), (bih, bil) = split(br), split(bi)
        terms = [(arh, aih, brh, bih), (arh, aih, brl, bil), (arl, ail, brh, bih)]
        if lolo:
            terms.append((arl, ail, brl, bil))
        sr = sum(x.T @ y + u.T @ v for x, u, y, v in terms)
        si = sum(x.T @ v - u.T @ y for x, u, y, v in terms)
    return -(sr + 1j * si)


def sigx_model(blocks, nqp, path="bf16x3"):
    """blocks: (Z complex64 [nocc, nmu, nqp], v [nmu], wk) of Eq.(sigx)."""
    out = np.zeros((nqp, nqp), np.complex128)
    for z, v, wk in blocks:
        nocc, nmu, _ = z.shape
        out += weighted_model(np.asarray(z).reshape(nocc * nmu, nqp),
                              np.tile(np.asarray(v, np.float64) * wk, nocc), path)
    return mirror_lower(out)


def chi0_model(blocks, npb, omega, delta_min, path="bf16x3", lolo=False):
    """blocks: (Z complex64 [nocc, nunocc, npb], eps_occ, eps_unocc, wk)."""
    out = np.zeros((len(omega), npb, npb), np.complex128)
    for z, eo, eu, wk in blocks:
        nocc, nunocc, _ = z.shape
        a = np.asarray(z, np.complex64).reshape(nocc * nunocc, npb)
        d = oracle.pair_delta(eo, eu).reshape(-1)
        keep = oracle.pair_included(d, delta_min)
        for iw, w in enumerate(omega):
            c = np.where(keep, -oracle.transition_weight(np.where(keep, d, 1.0), float(w), wk), 0.0)
            c32 = c.astype(np.float32)[:, None]
            br = (a.real.astype(np.float32) * c32).astype(np.float32)
            bi = (a.imag.astype(np.float32) * c32).astype(np.float32)
            ar = a.real.astype(np.float32)
            ai = a.imag.astype(np.float32)
            if path == "fp32":
                ar64, ai64, br64, bi64 = (x.astype(np.float64) for x in (ar, ai, br, bi))
                sr = ar64.T @ br64 + ai64.T @ bi64
                si = ar64.T @ bi64 - ai64.T @ br64
            else:
                (arh, arl), (aih, ail) = split(ar), split(ai)
                (brh, brl), (bih, bil) = split(br), split(bi)
                terms = [(arh, aih, brh, bih), (arh, aih, brl, bil), (arl, ail, brh, bih)]
                if lolo:
                    terms.append((arl, ail, brl, bil))
                sr = sum(x.T @ y + u.T @ v for x, u, y, v in terms)
                si = sum(x.T @ v - u.T @ y for x, u, y, v in terms)
            out[iw] -= sr + 1j * si
    return mirror_lower(out)


def hist_model(blocks, npb, edges, sigma, delta_min=0.0, path="bf16x3", lolo=False):
    """Histogram bins of the reduced-precision path: per bin, the weighted
    rank-K model over the pairs with a non-zero bin weight (FP32 weight on
    the Q side, bf16 split); blocks: (Z complex64 [nocc, nunocc, npb], eps_occ,
    eps_unocc, wk)."""
    from oracle.hist_oracle import pair_bin_table
    nb = len(edges) - 1
    out = np.zeros((nb, npb, npb), np.complex128)
    for z, eo, eu, wk in blocks:
        nocc, nunocc, _ = z.shape
        a = np.asarray(z, np.complex64).reshape(nocc * nunocc, npb)
        t = pair_bin_table(eo, eu, edges, sigma, delta_min, wk)
        for j in range(nb):
            rows = np.nonzero(t[j])[0]
            if rows.size:
                out[j] += weighted_model(a[rows], t[j, rows], path, lolo)
    return mirror_lower(out)


def sigc_model(blocks, eps_qp, mesh):
    """I^c with both contractions on BF16x3 as the GPU runs them: W^c
    rounded to FP32 and split into bf16 hi / lo; Z multiplied by the
    integration weight of its column and mesh point in FP64, rounded to FP32
    and split; three split products per real product summed exactly (FP64)
    over all (mesh point, mu) rows; the second contraction the same way on
    zw and Z rounded to FP32 and split.
    blocks: (Z [nall, nmu, nqp], W^c [nomega, nmu, nmu], eps_mid, wk)."""
    from oracle.sigc_oracle import ag_weight_table
    nqp = len(eps_qp)
    out = np.zeros((nqp, nqp), np.complex128)
    for z, wc, eps_mid, wk in blocks:
        z = np.asarray(z, np.complex128)
        wc = np.asarray(wc, np.complex128)
        t = -float(wk) * ag_weight_table(eps_qp, eps_mid, mesh)       # [n', n, i]
        wsplit = []
        for i in range(wc.shape[0]):
            wr32, wi32 = wc[i].real.astype(np.float32), wc[i].imag.astype(np.float32)
            wsplit.append((split(wr32), split(wi32)))
        for a in range(z.shape[0]):
            zw = np.zeros((wc.shape[1], nqp), np.complex128)           # D[nu][n]
            for i in range(wc.shape[0]):
                (wrh, wrl), (wih, wil) = wsplit[i]
                ti = t[a, :, i][None, :]
                (zrh, zrl) = split((z[a].real * ti).astype(np.float32))
                (zih, zil) = split((z[a].imag * ti).astype(np.float32))
                for (pr, pi), (qr, qi) in (((wrh, wih), (zrh, zih)), ((wrh, wih), (zrl, zil)),
                                           ((wrl, wil), (zrh, zih))):
                    zw += (pr.T @ qr + pi.T @ qi) + 1j * (pr.T @ qi - pi.T @ qr)
            (awrh, awrl), (awih, awil) = split(zw.real.astype(np.float32)), split(zw.imag.astype(np.float32))
            (bzrh, bzrl), (bzih, bzil) = (split(z[a].real.astype(np.float32)),
                                          split(z[a].imag.astype(np.float32)))
            for (pr, pi), (qr, qi) in (((awrh, awih), (bzrh, bzih)), ((awrh, awih), (bzrl, bzil)),
                                       ((awrl, awil), (bzrh, bzih))):
                out += (pr.T @ qr + pi.T @ qi) + 1j * (pr.T @ qi - pi.T @ qr)
    return out
