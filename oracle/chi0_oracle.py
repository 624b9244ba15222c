"""CPU FP64 oracle for the polarization chi0(q, i omega) and the dielectric step.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call this module.  The GPU
library never uses it, and it shares no code with the GPU path; its inputs
come from the seeded generator in ``synth/`` only.

What it computes (all complex128 / float64):

* Transition weight.  The time-reversal-symmetric polarization, Eq.(polfx),
  weights each occupied -> unoccupied pair (n, n') with
  1/(w - D + i0) - 1/(w + D - i0),  D = eps_{q+k,n'} - eps_{k,n}.
  On the imaginary axis w -> i*omega the infinitesimals can be dropped (the
  text below Eq.(polfx) says so), and
  1/(i omega - D) - 1/(i omega + D) = -2 D / (D^2 + omega^2).
  Each block additionally carries a k-point weight w_k (normalisation of the
  bare Brillouin-zone sum).
* chi0[I, J] = sum_blocks w_k sum_{n occ} sum_{n' unocc, pair included}
               f(D, omega) conj(Z_{nn'}(I)) Z_{nn'}(J),
  conjugation on the first basis index, as in the GEMM Z_pair^dagger x W_Zpair
  of Algorithm "hrcxq" (the printed Eq.(polfx) conjugates the second index;
  the two conventions are transposes of each other since chi0 is Hermitian).
  A pair is included iff D > 0 and D >= delta_min.  A pair with D <= 0 (an
  "unoccupied" state at or below an occupied one) is not a transition of
  Eq.(polfx); such input is rejected (``InvalidPairs``) unless the caller
  asks for it to be skipped (``strict=False``).
* eps[I, J] = delta_IJ - s_I chi0[I, J] s_J with s_I = sqrt(v_I),
  Eq.(dielectricfunction).
* eps^{-1}: Gauss-Jordan elimination with partial pivoting on [eps | 1]
  (textbook), the Cholesky route for Hermitian positive definite eps
  (eps = L L^H, then L Y = 1 and L^H X = Y by substitution; eps is HPD
  because chi0 is negative semidefinite), or LAPACK's inverse as a library
  primitive for large matrices.
* W^c[I, J] = s_I (eps^{-1} - 1)[I, J] s_J, Eq.(wc).

Parity pins for every function live in ``tests/pins.py`` (run by
``tests/test_oracle_pins.py``); none of the functions here is "parity
unpinned".
"""
from __future__ import annotations

from fractions import Fraction
from typing import Iterable, Iterator, List, Optional, Sequence, Tuple

import numpy as np

# ---------------------------------------------------------------------------
# Transition weights (Eq.(polfx) on the imaginary axis)
# ---------------------------------------------------------------------------


def pair_delta(eps_occ: np.ndarray, eps_unocc: np.ndarray) -> np.ndarray:
    """D[n, n'] = eps_unocc[n'] - eps_occ[n] (float64), Eq.(polfx)."""
    return np.asarray(eps_unocc, np.float64)[None, :] - np.asarray(eps_occ, np.float64)[:, None]


def pair_included(delta: np.ndarray, delta_min: float) -> np.ndarray:
    """Pairs that enter the sum: positive excitation energy at or above the
    intraband cut delta_min."""
    return (delta > 0.0) & (delta >= delta_min)


class InvalidPairs(ValueError):
    """Some pair has D = eps_unocc - eps_occ <= 0."""


def nonpositive_pairs(eps_occ: np.ndarray, eps_unocc: np.ndarray) -> int:
    """Number of pairs with D <= 0 (input the polarization sum does not
    define: every transition of Eq.(polfx) has a positive energy)."""
    return int(np.count_nonzero(~(pair_delta(eps_occ, eps_unocc) > 0.0)))


def _check_pairs(eps_occ, eps_unocc, strict: bool) -> None:
    if strict:
        bad = nonpositive_pairs(eps_occ, eps_unocc)
        if bad:
            raise InvalidPairs(f"{bad} pair(s) with D <= 0")


def transition_weight(delta: np.ndarray, omega: float, wk: float) -> np.ndarray:
    """w_k * (1/(i omega - D) - 1/(i omega + D)) = -2 w_k D / (D^2 + omega^2)."""
    delta = np.asarray(delta, np.float64)
    return -2.0 * wk * delta / (delta * delta + omega * omega)


# ---------------------------------------------------------------------------
# chi0, reference tier: per-block matrix products in FP64, blocks combined
# with compensated (two-sum) addition.
# ---------------------------------------------------------------------------


def _two_sum(a: np.ndarray, b: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    s = a + b
    bp = s - a
    e = (a - (s - bp)) + (b - bp)
    return s, e


class _CompensatedSum:
    """Running sum of complex arrays with Knuth two-sum error terms on the
    real and imaginary parts separately."""

    def __init__(self, shape):
        self.re = np.zeros(shape)
        self.im = np.zeros(shape)
        self.ce = np.zeros(shape)
        self.ci = np.zeros(shape)

    def add(self, x: np.ndarray) -> None:
        self.re, e = _two_sum(self.re, x.real)
        self.ce += e
        self.im, e = _two_sum(self.im, x.imag)
        self.ci += e

    def value(self) -> np.ndarray:
        return (self.re + self.ce) + 1j * (self.im + self.ci)


BlockInput = Tuple[np.ndarray, np.ndarray, np.ndarray, float]
# (Z[nocc, nunocc, npb] complex, eps_occ[nocc], eps_unocc[nunocc], w_k)


def chi0_block(z: np.ndarray, eps_occ: np.ndarray, eps_unocc: np.ndarray,
               wk: float, omega: Sequence[float], delta_min: float,
               strict: bool = True) -> np.ndarray:
    """Contribution of one block: [nomega, npb, npb] complex128."""
    _check_pairs(eps_occ, eps_unocc, strict)
    z = np.asarray(z)
    nocc, nunocc, npb = z.shape
    a = z.reshape(nocc * nunocc, npb).astype(np.complex128)
    delta = pair_delta(eps_occ, eps_unocc).reshape(-1)
    keep = pair_included(delta, delta_min)
    a = a[keep]
    delta = delta[keep]
    out = np.empty((len(omega), npb, npb), np.complex128)
    for iw, w in enumerate(omega):
        c = transition_weight(delta, float(w), wk)          # [K]
        out[iw] = a.conj().T @ (c[:, None] * a)              # sum_K conj(Z_I) c Z_J
    return out


def chi0_ref(blocks: Iterable[BlockInput], npb: int, omega: Sequence[float],
             delta_min: float = 0.0, strict: bool = True) -> np.ndarray:
    """chi0[nomega, npb, npb] for one q-point, streaming over blocks."""
    acc = _CompensatedSum((len(omega), npb, npb))
    for z, eo, eu, wk in blocks:
        acc.add(chi0_block(z, eo, eu, wk, omega, delta_min, strict))
    return acc.value()


def chi0_ref_per_block(blocks: Iterable[BlockInput], npb: int,
                       omega: Sequence[float], delta_min: float = 0.0,
                       strict: bool = True) -> List[np.ndarray]:
    """Per-block contributions (for additivity / per-spin diagnostics)."""
    return [chi0_block(z, eo, eu, wk, omega, delta_min, strict) for z, eo, eu, wk in blocks]


# ---------------------------------------------------------------------------
# chi0, brute-force tier: explicit loops (tiny inputs only)
# ---------------------------------------------------------------------------


def chi0_brute(blocks: Iterable[BlockInput], npb: int, omega: Sequence[float],
               delta_min: float = 0.0, strict: bool = True) -> np.ndarray:
    out = np.zeros((len(omega), npb, npb), np.complex128)
    for z, eo, eu, wk in blocks:
        _check_pairs(eo, eu, strict)
        nocc, nunocc, _ = np.shape(z)
        for iw, w in enumerate(omega):
            for n in range(nocc):
                for m in range(nunocc):
                    d = float(eu[m]) - float(eo[n])
                    if not (d > 0.0 and d >= delta_min):
                        continue
                    f = -2.0 * wk * d / (d * d + float(w) * float(w))
                    for i in range(npb):
                        zi = complex(z[n][m][i]).conjugate()
                        for j in range(npb):
                            out[iw, i, j] += f * zi * complex(z[n][m][j])
    return out


# ---------------------------------------------------------------------------
# chi0, exact tier: rational arithmetic (small integer Z, dyadic energies)
# ---------------------------------------------------------------------------


def chi0_exact(blocks, npb: int, omega: Sequence[Fraction],
               delta_min: Fraction = Fraction(0), strict: bool = True):
    """Exact chi0 with Fractions.  Z entries are (re, im) pairs of Fractions;
    energies, w_k and omega are Fractions.  Returns nested lists
    [iw][I][J] of (re, im) Fraction pairs."""
    res = [[[(Fraction(0), Fraction(0)) for _ in range(npb)] for _ in range(npb)]
           for _ in omega]
    for z, eo, eu, wk in blocks:
        if strict and any(not (u - o > 0) for o in eo for u in eu):
            raise InvalidPairs("pair(s) with D <= 0")
        for iw, w in enumerate(omega):
            for n in range(len(eo)):
                for m in range(len(eu)):
                    d = eu[m] - eo[n]
                    if not (d > 0 and d >= delta_min):
                        continue
                    f = -2 * wk * d / (d * d + w * w)
                    for i in range(npb):
                        ar, ai = z[n][m][i]
                        for j in range(npb):
                            br, bi = z[n][m][j]
                            # conj(a) * b = (ar - i ai)(br + i bi)
                            re = ar * br + ai * bi
                            im = ar * bi - ai * br
                            cr, ci = res[iw][i][j]
                            res[iw][i][j] = (cr + f * re, ci + f * im)
    return res


# ---------------------------------------------------------------------------
# chi0 rows (full-size checks of whole rows)
# ---------------------------------------------------------------------------


def chi0_rows(blocks: Iterable[BlockInput], rows: Sequence[int], npb: int,
              omega: Sequence[float], delta_min: float = 0.0,
              strict: bool = True) -> np.ndarray:
    """chi0[iw, I, :] for the listed rows I only, [nomega, len(rows), npb]:
    sum over pairs of f conj(Z(I)) Z(J) for every J, blocks combined with
    compensated sums (the reference tier restricted to some rows)."""
    rows = np.asarray(rows, dtype=np.int64)
    acc = _CompensatedSum((len(omega), len(rows), npb))
    for z, eo, eu, wk in blocks:
        _check_pairs(eo, eu, strict)
        z = np.asarray(z)
        nocc, nunocc, _ = z.shape
        a = z.reshape(nocc * nunocc, npb).astype(np.complex128)
        delta = pair_delta(eo, eu).reshape(-1)
        keep = pair_included(delta, delta_min)
        a = a[keep]
        delta = delta[keep]
        part = np.empty((len(omega), len(rows), npb), np.complex128)
        for iw, w in enumerate(omega):
            c = transition_weight(delta, float(w), wk)
            part[iw] = (a[:, rows].conj() * c[:, None]).T @ a
        acc.add(part)
    return acc.value()


# ---------------------------------------------------------------------------
# chi0 entries one by one (full-size spot checks)
# ---------------------------------------------------------------------------


def chi0_entries(block_columns: Iterable[Tuple[np.ndarray, np.ndarray, np.ndarray, float]],
                 entries: Sequence[Tuple[int, int]], col_index: dict,
                 omega: Sequence[float], delta_min: float = 0.0,
                 strict: bool = True) -> np.ndarray:
    """chi0[iw, I, J] for the listed (I, J) entries only.

    ``block_columns`` yields (Zc[K, ncols], eps_occ, eps_unocc, w_k) where Zc
    holds the columns of Z (pairs flattened n-major) listed in ``col_index``
    (basis index -> column of Zc).  Returns [nomega, len(entries)]."""
    acc = _CompensatedSum((len(omega), len(entries)))
    ii = np.array([col_index[i] for i, _ in entries])
    jj = np.array([col_index[j] for _, j in entries])
    for zc, eo, eu, wk in block_columns:
        _check_pairs(eo, eu, strict)
        delta = pair_delta(eo, eu).reshape(-1)
        keep = pair_included(delta, delta_min)
        zc = np.asarray(zc, np.complex128)[keep]
        delta = delta[keep]
        part = np.empty((len(omega), len(entries)), np.complex128)
        for iw, w in enumerate(omega):
            c = transition_weight(delta, float(w), wk)
            part[iw] = np.sum(c[:, None] * zc[:, ii].conj() * zc[:, jj], axis=0)
        acc.add(part)
    return acc.value()


# ---------------------------------------------------------------------------
# Dielectric matrix, inverse, W^c
# ---------------------------------------------------------------------------


def dielectric(chi0: np.ndarray, vsqrt: np.ndarray) -> np.ndarray:
    """eps = 1 - s chi0 s (per frequency), Eq.(dielectricfunction)."""
    chi0 = np.asarray(chi0, np.complex128)
    s = np.asarray(vsqrt, np.float64)
    npb = s.shape[0]
    return np.eye(npb)[None] - s[None, :, None] * chi0 * s[None, None, :]


def inverse_gauss_jordan(a: np.ndarray) -> np.ndarray:
    """Textbook Gauss-Jordan inversion with partial (row) pivoting on [a | 1].
    The pivot is the entry of largest modulus in the current column."""
    a = np.array(a, dtype=np.complex128)
    n = a.shape[0]
    aug = np.concatenate([a, np.eye(n, dtype=np.complex128)], axis=1)
    for k in range(n):
        p = k + int(np.argmax(np.abs(aug[k:, k])))
        if aug[p, k] == 0:
            raise np.linalg.LinAlgError("singular matrix")
        if p != k:
            aug[[k, p]] = aug[[p, k]]
        aug[k] = aug[k] / aug[k, k]
        col = aug[:, k].copy()
        col[k] = 0.0
        aug -= col[:, None] * aug[k][None, :]
    return aug[:, n:]


class NotHPD(np.linalg.LinAlgError):
    """A Cholesky pivot was not positive: the matrix is not Hermitian
    positive definite (numerically)."""


def cholesky_lower(a: np.ndarray) -> np.ndarray:
    """Textbook column-by-column Cholesky factor L (lower, real positive
    diagonal) with a = L L^H, reading only the lower triangle of a."""
    a = np.array(a, dtype=np.complex128)
    n = a.shape[0]
    low = np.zeros_like(a)
    for j in range(n):
        d = a[j, j].real - np.sum(np.abs(low[j, :j]) ** 2)
        if not d > 0.0:
            raise NotHPD(f"pivot {j} = {d}")
        low[j, j] = np.sqrt(d)
        low[j + 1:, j] = (a[j + 1:, j] - low[j + 1:, :j] @ low[j, :j].conj()) / low[j, j]
    return low


def inverse_cholesky(a: np.ndarray) -> np.ndarray:
    """Inverse of a Hermitian positive definite matrix via a = L L^H: forward
    substitution L Y = 1, then back substitution L^H X = Y."""
    low = cholesky_lower(a)
    n = low.shape[0]
    y = np.zeros((n, n), np.complex128)
    eye = np.eye(n, dtype=np.complex128)
    for i in range(n):
        y[i] = (eye[i] - low[i, :i] @ y[:i]) / low[i, i]
    up = low.conj().T
    x = np.zeros((n, n), np.complex128)
    for i in range(n - 1, -1, -1):
        x[i] = (y[i] - up[i, i + 1:] @ x[i + 1:]) / up[i, i]
    return x


def inverse(eps: np.ndarray, method: str = "gauss_jordan") -> np.ndarray:
    """Inverse of each frequency's matrix; eps is [nomega, n, n] or [n, n]."""
    eps = np.asarray(eps, np.complex128)
    single = eps.ndim == 2
    if single:
        eps = eps[None]
    if method == "gauss_jordan":
        out = np.stack([inverse_gauss_jordan(e) for e in eps])
    elif method == "cholesky":
        out = np.stack([inverse_cholesky(e) for e in eps])
    elif method == "lapack":
        out = np.linalg.inv(eps)
    else:
        raise ValueError(method)
    return out[0] if single else out


def screened_wc(eps_inv: np.ndarray, vsqrt: np.ndarray) -> np.ndarray:
    """W^c = s (eps^{-1} - 1) s, Eq.(wc)."""
    s = np.asarray(vsqrt, np.float64)
    npb = s.shape[0]
    d = np.asarray(eps_inv, np.complex128) - np.eye(npb)
    return s[..., :, None] * d * s[..., None, :] if d.ndim == 2 else \
        s[None, :, None] * d * s[None, None, :]


# ---------------------------------------------------------------------------
# Convenience: oracle over a synthetic workload
# ---------------------------------------------------------------------------


def workload_blocks(wl, q: int = 0, blocks=None) -> Iterator[BlockInput]:
    """Stream (Z, eps_occ, eps_unocc, w_k) for a synthetic workload."""
    for blk in (wl.blocks(q) if blocks is None else blocks):
        eo, eu = wl.energies(blk)
        yield wl.z_block(blk), eo, eu, blk.wk


def chi0_workload(wl, q: int = 0, blocks=None) -> np.ndarray:
    return chi0_ref(workload_blocks(wl, q, blocks), wl.npb, wl.omega, wl.delta_min)


def rel_fro(x: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-frequency relative Frobenius error ||x - ref||_F / ||ref||_F."""
    x = np.asarray(x)
    ref = np.asarray(ref)
    if ref.ndim == 2:
        return np.linalg.norm(x - ref) / np.linalg.norm(ref)
    num = np.linalg.norm((x - ref).reshape(ref.shape[0], -1), axis=1)
    den = np.linalg.norm(ref.reshape(ref.shape[0], -1), axis=1)
    return num / den
