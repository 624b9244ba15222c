"""Pins for the CPU oracle: checks against what the mathematics fixes, written
independently of the oracle's own code.

Each pin takes the oracle module and returns a list of failure messages (empty
when the pin holds), so that ``test_oracle_mutations.py`` can plant a mistake
in the oracle and show that at least one pin catches it.
"""
from __future__ import annotations

import json
import os
from fractions import Fraction

import numpy as np

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
U = np.finfo(np.float64).eps / 2


def _frac_mat(m):
    return np.array([[complex(float(Fraction(re)), float(Fraction(im))) for re, im in row]
                     for row in m])


def _load_golden():
    with open(os.path.join(GOLDEN, "two_basis_example.json")) as f:
        g = json.load(f)
    z = np.array([[[complex(float(Fraction(a)), float(Fraction(b))) for a, b in vec]
                   for vec in occ] for occ in g["z"]])
    eo = np.array([float(Fraction(x)) for x in g["eps_occ"]])
    eu = np.array([float(Fraction(x)) for x in g["eps_unocc"]])
    wk = float(Fraction(g["wk"]))
    s = np.array([float(Fraction(x)) for x in g["vsqrt"]])
    return g, z, eo, eu, wk, s


def _close(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


def pin_golden(orc):
    """Hand-derived two-basis example (tests/golden/two_basis_example.json)."""
    fails = []
    g, z, eo, eu, wk, s = _load_golden()
    for case in g["cases"]:
        w = float(Fraction(case["omega"]))
        dmin = float(Fraction(case["delta_min"]))
        chi = orc.chi0_ref([(z, eo, eu, wk)], 2, [w], dmin)[0]
        if not _close(chi, _frac_mat(case["chi0"]), 1e-15):
            fails.append(f"golden chi0 omega={w} dmin={dmin}: {chi}")
        if "eps" in case:
            eps = orc.dielectric(chi[None], s)[0]
            if not _close(eps, _frac_mat(case["eps"]), 1e-15):
                fails.append(f"golden eps: {eps}")
            for method in ("gauss_jordan", "cholesky", "lapack"):
                inv = orc.inverse(eps, method)
                if not _close(inv, _frac_mat(case["eps_inv"]), 1e-15):
                    fails.append(f"golden eps_inv ({method}): {inv}")
            wc = orc.screened_wc(orc.inverse(eps), s)
            if not _close(wc, _frac_mat(case["wc"]), 1e-15):
                fails.append(f"golden wc: {wc}")
    return fails


def pin_weight_is_polfx_on_imaginary_axis(orc):
    """The weight equals the bracket of Eq.(polfx), 1/(w - D) - 1/(w + D),
    evaluated with complex arithmetic at w = i*omega (the +-i0 dropped)."""
    fails = []
    for d in (1e-3, 0.05, 0.7, 3.0):
        for w in (0.0, 1e-2, 0.3, 2.0, 50.0):
            for wk in (1.0, 0.125):
                z = 1j * w
                ref = wk * (1.0 / (z - d) - 1.0 / (z + d))
                got = float(orc.transition_weight(np.array([d]), w, wk)[0])
                if abs(ref.imag) > 1e-14 * abs(ref) or abs(got - ref.real) > 4 * U * abs(ref):
                    fails.append(f"weight D={d} omega={w}: {got} vs {ref}")
    return fails


def _small_int_problem(rng, nblocks=2, nocc=2, nunocc=3, npb=3):
    """Small-integer Z, dyadic energies (exact in binary floating point)."""
    blocks_f, blocks_q = [], []
    for b in range(nblocks):
        zr = rng.integers(-3, 4, size=(nocc, nunocc, npb))
        zi = rng.integers(-3, 4, size=(nocc, nunocc, npb))
        eo = -rng.integers(1, 8, size=nocc) / 8.0
        eu = rng.integers(0, 16, size=nunocc) / 8.0
        wk = 1.0 / nblocks
        blocks_f.append((zr + 1j * zi, eo, eu, wk))
        zq = [[[(Fraction(int(zr[n, m, i])), Fraction(int(zi[n, m, i]))) for i in range(npb)]
               for m in range(nunocc)] for n in range(nocc)]
        blocks_q.append((zq, [Fraction(x).limit_denominator(8) for x in eo],
                         [Fraction(x).limit_denominator(8) for x in eu], Fraction(1, nblocks)))
    return blocks_f, blocks_q


def pin_exact_bruteforce(orc):
    """Exact rational brute force == FP64 reference == FP64 loops (tiny)."""
    fails = []
    rng = np.random.default_rng(11)
    omega_f = [0.0, 0.5, 2.0]
    omega_q = [Fraction(0), Fraction(1, 2), Fraction(2)]
    for dmin_f, dmin_q in ((0.0, Fraction(0)), (0.5, Fraction(1, 2))):
        bf, bq = _small_int_problem(rng)
        ex = orc.chi0_exact(bq, 3, omega_q, dmin_q)
        exact = np.array([[[complex(float(r), float(i)) for r, i in row] for row in m] for m in ex])
        ref = orc.chi0_ref(bf, 3, omega_f, dmin_f)
        brute = orc.chi0_brute(bf, 3, omega_f, dmin_f)
        for name, x in (("ref", ref), ("brute", brute)):
            err = np.max(np.abs(x - exact)) / max(np.max(np.abs(exact)), 1e-300)
            if not err <= 1e-15:
                fails.append(f"exact vs {name}, dmin={dmin_f}: {err}")
    return fails


def pin_conjugation_side(orc):
    """One pair, Z = [1, i]: chi0[0, 1] = f * conj(1) * i = i f (conjugate on
    the first index, Algorithm "hrcxq" GEMM Z_pair^dagger x W_Zpair)."""
    z = np.array([[[1.0 + 0j, 1j]]])
    chi = orc.chi0_ref([(z, np.array([-0.5]), np.array([0.5]), 1.0)], 2, [1.0])[0]
    f = -2.0 * 1.0 / (1.0 + 1.0)
    if not _close(chi, np.array([[f, 1j * f], [-1j * f, f]]), 1e-15):
        return [f"conjugation side: {chi}"]
    return []


def pin_single_transition(orc):
    """Rank one: chi0 = w f conj(z) z^T; eps^-1 by Sherman-Morrison;
    W^c = -g s a a^H s / (1 + g |a|^2) with a = s * conj(z), g = -w f."""
    fails = []
    rng = np.random.default_rng(3)
    npb = 6
    z = rng.standard_normal(npb) + 1j * rng.standard_normal(npb)
    s = 1.0 / (1.0 + np.arange(npb))
    eo, eu, wk = np.array([-0.3]), np.array([0.45]), 0.25
    d = 0.75
    for w in (0.0, 0.2, 3.0):
        f = -2.0 * d / (d * d + w * w)
        chi = orc.chi0_ref([(z.reshape(1, 1, npb), eo, eu, wk)], npb, [w])[0]
        ref = wk * f * np.outer(z.conj(), z)
        if not _close(chi, ref, 4e-15):
            fails.append(f"single transition chi0 omega={w}")
        g = -wk * f
        a = s * z.conj()
        eps = orc.dielectric(chi[None], s)[0]
        if not _close(eps, np.eye(npb) + g * np.outer(a, a.conj()), 4e-15):
            fails.append(f"single transition eps omega={w}")
        inv_ref = np.eye(npb) - g * np.outer(a, a.conj()) / (1.0 + g * np.vdot(a, a).real)
        for method in ("gauss_jordan", "cholesky", "lapack"):
            inv = orc.inverse(eps, method)
            if not _close(inv, inv_ref, 1e-14):
                fails.append(f"single transition eps_inv {method} omega={w}")
        wc = orc.screened_wc(orc.inverse(eps), s)
        if not _close(wc, s[:, None] * (inv_ref - np.eye(npb)) * s[None, :], 1e-14):
            fails.append(f"single transition wc omega={w}")
    return fails


def _random_problem(rng, nblocks=3, nocc=4, nunocc=9, npb=7, dmin_gap=0.02):
    blocks = []
    for _ in range(nblocks):
        z = rng.standard_normal((nocc, nunocc, npb)) + 1j * rng.standard_normal((nocc, nunocc, npb))
        z *= np.exp(-np.arange(npb) / 4.0)
        eo = rng.uniform(-0.8, 0.0, nocc)
        eu = rng.uniform(dmin_gap, 3.0, nunocc)
        blocks.append((z, eo, eu, 1.0 / nblocks))
    return blocks


def pin_invariants(orc):
    """Hermitian, negative semidefinite (text below Eq.(polfx)), even in omega,
    Loewner-monotone in omega, rank <= number of pairs, eps >= 1 and
    eps^-1 eigenvalues in (0, 1], W^c <= 0."""
    fails = []
    rng = np.random.default_rng(5)
    npb = 9
    blocks = _random_problem(rng, npb=npb)
    omega = [0.0, 0.05, 0.3, 1.0, 4.0]
    chi = orc.chi0_ref(blocks, npb, omega)
    chin = orc.chi0_ref(blocks, npb, [-w for w in omega])
    s = 1.0 / (1.0 + np.arange(npb))
    for iw in range(len(omega)):
        c = chi[iw]
        nrm = np.linalg.norm(c)
        if np.max(np.abs(c - c.conj().T)) > 1e-14 * nrm:
            fails.append(f"hermitian iw={iw}")
        ev = np.linalg.eigvalsh(0.5 * (c + c.conj().T))
        if ev.max() > 64 * U * nrm:
            fails.append(f"NSD iw={iw}: max eig {ev.max()}")
        if np.max(np.abs(chin[iw] - c)) > 4 * U * nrm:
            fails.append(f"even in omega iw={iw}")
        if iw:
            dd = chi[iw] - chi[iw - 1]
            if np.linalg.eigvalsh(0.5 * (dd + dd.conj().T)).min() < -64 * U * nrm:
                fails.append(f"Loewner monotone iw={iw}")
        eps = orc.dielectric(c[None], s)[0]
        eve = np.linalg.eigvalsh(0.5 * (eps + eps.conj().T))
        if eve.min() < 1.0 - 1e-12:
            fails.append(f"eps >= 1 iw={iw}: {eve.min()}")
        inv = orc.inverse(eps)
        evi = np.linalg.eigvalsh(0.5 * (inv + inv.conj().T))
        if evi.min() <= 0 or evi.max() > 1.0 + 1e-12:
            fails.append(f"eps_inv spectrum iw={iw}: {evi.min()} {evi.max()}")
        wc = orc.screened_wc(inv, s)
        if np.linalg.eigvalsh(0.5 * (wc + wc.conj().T)).max() > 1e-12:
            fails.append(f"W^c <= 0 iw={iw}")
    # rank <= K: 2 pairs in npb = 9
    z = rng.standard_normal((1, 2, npb)) + 1j * rng.standard_normal((1, 2, npb))
    c = orc.chi0_ref([(z, np.array([-0.1]), np.array([0.2, 0.9]), 1.0)], npb, [0.3])[0]
    ev = np.sort(np.abs(np.linalg.eigvalsh(c)))
    if ev[-3] > 1e-13 * ev[-1]:
        fails.append(f"rank <= K: {ev}")
    return fails


def pin_large_omega_tail(orc):
    """T = -2 sum w_k D conj(Z) Z^T (the 1/omega^2 coefficient).  For every
    omega: 0 <= omega^2 chi0 - T <= Dmax^2/(Dmax^2 + omega^2) (-T) (Loewner)."""
    fails = []
    rng = np.random.default_rng(9)
    npb = 8
    blocks = _random_problem(rng, npb=npb)
    tail = np.zeros((npb, npb), complex)
    dmax = 0.0
    for z, eo, eu, wk in blocks:
        for n in range(z.shape[0]):
            for m in range(z.shape[1]):
                d = eu[m] - eo[n]
                dmax = max(dmax, d)
                tail += -2.0 * wk * d * np.outer(z[n, m].conj(), z[n, m])
    nrm = np.linalg.norm(tail)
    for w in (0.5, 10.0, 1e3, 1e4):
        c = orc.chi0_ref(blocks, npb, [w])[0]
        gap = w * w * c - tail
        lo = np.linalg.eigvalsh(0.5 * (gap + gap.conj().T)).min()
        up = (dmax ** 2 / (dmax ** 2 + w * w)) * (-tail) - gap
        hi = np.linalg.eigvalsh(0.5 * (up + up.conj().T)).min()
        if lo < -1e-12 * nrm or hi < -1e-12 * nrm:
            fails.append(f"tail bounds omega={w}: {lo} {hi}")
    return fails


def pin_structure(orc):
    """Additivity over blocks; invariance under permutations of n and n' and
    of blocks, and under per-pair phases; |alpha|^2 scaling; pairs below
    delta_min contribute exactly nothing."""
    fails = []
    rng = np.random.default_rng(21)
    npb = 6
    blocks = _random_problem(rng, npb=npb, nblocks=3)
    omega = [0.1, 1.5]
    full = orc.chi0_ref(blocks, npb, omega)
    parts = sum(orc.chi0_ref([b], npb, omega) for b in blocks)
    nrm = np.linalg.norm(full)
    if np.linalg.norm(full - parts) > 1e-14 * nrm:
        fails.append("additivity")
    if np.linalg.norm(orc.chi0_ref(blocks[::-1], npb, omega) - full) > 1e-14 * nrm:
        fails.append("block permutation")
    perm = []
    for z, eo, eu, wk in blocks:
        po = rng.permutation(z.shape[0])
        pu = rng.permutation(z.shape[1])
        ph = np.exp(1j * rng.uniform(0, 2 * np.pi, size=z.shape[:2]))[..., None]
        perm.append((z[po][:, pu] * ph, eo[po], eu[pu], wk))
    if np.linalg.norm(orc.chi0_ref(perm, npb, omega) - full) > 1e-14 * nrm:
        fails.append("pair permutation / phase")
    alpha = 0.7 - 1.3j
    scaled = [(alpha * z, eo, eu, wk) for z, eo, eu, wk in blocks]
    if np.linalg.norm(orc.chi0_ref(scaled, npb, omega) - abs(alpha) ** 2 * full) > 1e-14 * nrm:
        fails.append("scaling")
    # add pairs below the cut: occupied state just under an unoccupied one
    dmin = 0.01
    extra = []
    for z, eo, eu, wk in blocks:
        z2 = np.concatenate([z, rng.standard_normal((1,) + z.shape[1:]) * (1 + 1j)], axis=0)
        eo2 = np.concatenate([eo, [eu.min() - 0.5 * dmin]])
        # the planted occupied state also makes pairs with D >= dmin to
        # higher unoccupied states; remove them by zeroing those rows of Z
        dd = eu - eo2[-1]
        z2[-1, dd >= dmin] = 0.0
        extra.append((z2, eo2, eu, wk))
    if np.linalg.norm(orc.chi0_ref(extra, npb, omega, dmin) - full) > 1e-14 * nrm:
        fails.append("excluded pairs contribute")
    return fails


def pin_inverse(orc):
    """Inverse: Gauss-Jordan, Cholesky and LAPACK agree; residual bounded by
    kappa*u; matrices that need pivoting (zero / tiny leading entry) are
    inverted exactly; permutation matrix inverse is its transpose; the
    Cholesky factor reproduces its matrix, an indefinite matrix is rejected
    and a complex 2x2 HPD matrix has its closed-form inverse."""
    fails = []
    p = np.array([[0, 1, 0], [0, 0, 1], [1, 0, 0]], complex)
    if not _close(orc.inverse(p, "gauss_jordan"), p.T, 0.0):
        fails.append("permutation inverse")
    a = np.array([[1e-18, 1.0], [1.0, 1.0]], complex)
    ref = np.array([[-1.0, 1.0], [1.0, 0.0]])  # exact inverse rounds to this
    if not _close(orc.inverse(a, "gauss_jordan"), ref, 1e-15):
        fails.append(f"pivoting needed: {orc.inverse(a, 'gauss_jordan')}")
    rng = np.random.default_rng(2)
    n = 40
    x = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    e = np.eye(n) + x @ x.conj().T * 50
    gj = orc.inverse(e, "gauss_jordan")
    la = orc.inverse(e, "lapack")
    kappa = np.linalg.cond(e)
    if np.linalg.norm(gj - la) / np.linalg.norm(la) > 64 * kappa * U:
        fails.append("GJ vs LAPACK")
    if np.linalg.norm(e @ gj - np.eye(n)) > 64 * n * kappa * U:
        fails.append("GJ residual")
    ch = orc.inverse(e, "cholesky")
    if np.linalg.norm(ch - la) / np.linalg.norm(la) > 64 * kappa * U:
        fails.append("Cholesky vs LAPACK")
    # the factor itself: L L^H reproduces e, L is lower with a positive diagonal
    low = orc.cholesky_lower(e)
    if np.linalg.norm(low @ low.conj().T - e) > 64 * n * U * np.linalg.norm(e):
        fails.append("Cholesky factor L L^H != e")
    if np.any(np.triu(low, 1) != 0) or np.any(np.diag(low).real <= 0) or \
            np.any(np.diag(low).imag != 0):
        fails.append("Cholesky factor shape")
    # an indefinite Hermitian matrix is rejected; a 2x2 HPD matrix with a
    # complex off-diagonal entry has the closed-form inverse
    # [[d, -b], [-conj(b), a]] / (a d - |b|^2)
    bad = np.array([[1.0, 2.0], [2.0, 1.0]], complex)
    try:
        orc.inverse(bad, "cholesky")
        fails.append("indefinite matrix accepted")
    except orc.NotHPD:
        pass
    a2 = np.array([[4.0, 1.0 + 2.0j], [1.0 - 2.0j, 3.0]])
    ref2 = np.array([[3.0, -1.0 - 2.0j], [-1.0 + 2.0j, 4.0]]) / 7.0
    if not _close(orc.inverse(a2, "cholesky"), ref2, 1e-15):
        fails.append(f"2x2 closed form: {orc.inverse(a2, 'cholesky')}")
    return fails


def pin_entries(orc):
    """Sampled entries (the full-size checks' oracle) against the hand-derived
    golden example, exact rational brute force and the loop tier.  The
    columns are handed over in a permuted order through the column map, the
    blocks have unequal w_k, a delta_min cut drops pairs, and (I, J) entries
    are asymmetric (I != J both ways), so the conjugation side, the column
    map, the cut and w_k all show."""
    fails = []
    # golden example: Z columns reversed, all four entries
    g, z, eo, eu, wk, s = _load_golden()
    ents = [(0, 0), (0, 1), (1, 0), (1, 1)]
    zc = z.reshape(-1, 2)[:, ::-1]
    for case in g["cases"]:
        w = float(Fraction(case["omega"]))
        dmin = float(Fraction(case["delta_min"]))
        got = orc.chi0_entries([(zc, eo, eu, wk)], ents, {0: 1, 1: 0}, [w], dmin)[0]
        ref = _frac_mat(case["chi0"])
        if not _close(got, np.array([ref[i, j] for i, j in ents]), 1e-15):
            fails.append(f"entries golden omega={w} dmin={dmin}: {got}")
    # exact rationals: small integer Z, dyadic energies, w_k 1/2, 1/4, 1/8
    rng = np.random.default_rng(17)
    bf, bq = _small_int_problem(rng, nblocks=3, nocc=2, nunocc=3, npb=4)
    wks = [Fraction(1, 2), Fraction(1, 4), Fraction(1, 8)]
    bf = [(zz, o, u, float(w)) for (zz, o, u, _), w in zip(bf, wks)]
    bq = [(zz, o, u, w) for (zz, o, u, _), w in zip(bq, wks)]
    cols = [3, 1, 2]
    col_index = {c: k for k, c in enumerate(cols)}
    ents = [(3, 1), (1, 3), (2, 2), (3, 3), (1, 2), (2, 1)]
    omega_f, omega_q = [0.0, 0.5, 2.0], [Fraction(0), Fraction(1, 2), Fraction(2)]
    for dmin_f, dmin_q in ((0.0, Fraction(0)), (0.5, Fraction(1, 2))):
        ex = orc.chi0_exact(bq, 4, omega_q, dmin_q)
        want = np.array([[complex(float(ex[iw][i][j][0]), float(ex[iw][i][j][1])) for i, j in ents]
                         for iw in range(len(omega_q))])
        bc = [(zz.reshape(-1, 4)[:, cols], o, u, w) for zz, o, u, w in bf]
        got = orc.chi0_entries(bc, ents, col_index, omega_f, dmin_f)
        err = np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300)
        if not err <= 1e-15:
            fails.append(f"entries vs exact, dmin={dmin_f}: {err}")
    # loop tier on a random problem with a cut that removes some pairs
    rng = np.random.default_rng(23)
    npb = 7
    blocks = _random_problem(rng, npb=npb, nblocks=3, dmin_gap=0.02)
    blocks = [(zz, o, u, w * (1 + b)) for b, (zz, o, u, w) in enumerate(blocks)]
    omega = [0.0, 0.3, 2.5]
    dmin = 0.4
    brute = orc.chi0_brute(blocks, npb, omega, dmin)
    ents = [(6, 0), (0, 6), (3, 4), (4, 3), (5, 5), (2, 6)]
    cols = [6, 0, 4, 3, 5, 2]
    col_index = {c: k for k, c in enumerate(cols)}
    bc = [(zz.reshape(-1, npb)[:, cols], o, u, w) for zz, o, u, w in blocks]
    got = orc.chi0_entries(bc, ents, col_index, omega, dmin)
    want = np.stack([brute[:, i, j] for i, j in ents], axis=1)
    if np.max(np.abs(got - want)) > 1e-14 * np.max(np.abs(brute)):
        fails.append("entries vs loops")
    # a D <= 0 pair is rejected
    try:
        orc.chi0_entries([(np.ones((2, 1)), np.array([0.1, -0.5]), np.array([0.1]), 1.0)],
                         [(0, 0)], {0: 0}, [1.0])
        fails.append("entries accepted a pair with D = 0")
    except orc.InvalidPairs:
        pass
    return fails


def pin_rows(orc):
    """Whole rows (the full-size row checks' oracle) against the golden
    example and the loop tier: rows given out of order, a delta_min cut,
    unequal w_k; row I of the result is chi0[I, :] (conjugation on I)."""
    fails = []
    g, z, eo, eu, wk, s = _load_golden()
    for case in g["cases"]:
        w = float(Fraction(case["omega"]))
        dmin = float(Fraction(case["delta_min"]))
        got = orc.chi0_rows([(z, eo, eu, wk)], [1, 0], 2, [w], dmin)[0]
        ref = _frac_mat(case["chi0"])
        if not _close(got, ref[[1, 0]], 1e-15):
            fails.append(f"rows golden omega={w} dmin={dmin}: {got}")
    rng = np.random.default_rng(29)
    npb = 8
    blocks = _random_problem(rng, npb=npb, nblocks=3)
    blocks = [(zz, o, u, w * (2.0 - 0.5 * b)) for b, (zz, o, u, w) in enumerate(blocks)]
    omega = [0.0, 0.7, 3.0]
    brute = orc.chi0_brute(blocks, npb, omega, 0.3)
    rows = [5, 0, 7, 2]
    got = orc.chi0_rows(blocks, rows, npb, omega, 0.3)
    if np.max(np.abs(got - brute[:, rows, :])) > 1e-14 * np.max(np.abs(brute)):
        fails.append("rows vs loops")
    return fails


ALL_PINS = [pin_golden, pin_weight_is_polfx_on_imaginary_axis, pin_exact_bruteforce,
            pin_conjugation_side, pin_single_transition, pin_invariants,
            pin_large_omega_tail, pin_structure, pin_inverse, pin_entries, pin_rows]


def run_all(orc):
    out = {}
    for p in ALL_PINS:
        try:
            out[p.__name__] = p(orc)
        except Exception as exc:  # a planted mistake may also raise
            out[p.__name__] = [f"raised {type(exc).__name__}: {exc}"]
    return out
