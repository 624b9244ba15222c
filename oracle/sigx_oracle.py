"""CPU FP64 oracle for the exchange self-energy Sigma^x (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or call this module; it shares no code with the GPU
library.

Eq.(sigx): for the q-point's quasiparticle states n, m,
  Sigma^x[n][m] = - sum_k w_k sum_{n' occ} sum_mu
                  conj(Z_k[n'][mu][n]) v_k[mu] Z_k[n'][mu][m],
with Z_k[n'][mu][n] the matrix element of Eq.(defz) between the product-basis
function mu of k and the states (q-k, n') and (q, n), v_k[mu] >= 0 the
Coulomb eigenvalues of Eq.(sigx), and w_k a per-k weight (1 for the bare
Brillouin-zone sum as printed; the caller may carry a 1/N_k normalisation
here).  Sigma^x is Hermitian and negative semidefinite.

Pins live in ``tests/pins_sigx.py``; none of these functions is "parity
unpinned".
"""
from __future__ import annotations

from fractions import Fraction
from typing import Iterable, Sequence, Tuple

import numpy as np

from .chi0_oracle import _CompensatedSum

SigxBlock = Tuple[np.ndarray, np.ndarray, float]
# (Z[nocc, nmu, nqp] complex, v[nmu] >= 0, w_k)


def sigx_block(z: np.ndarray, v: np.ndarray, wk: float) -> np.ndarray:
    """Contribution of one k-point: -w_k sum_{n', mu} conj(Z) v Z, [nqp, nqp]."""
    z = np.asarray(z)
    nocc, nmu, nqp = z.shape
    a = z.reshape(nocc * nmu, nqp).astype(np.complex128)        # rows (n', mu)
    c = np.tile(np.asarray(v, np.float64), nocc) * float(wk)      # v_mu per row
    return -(a.conj().T @ (c[:, None] * a))


def sigx_ref(blocks: Iterable[SigxBlock], nqp: int) -> np.ndarray:
    """Sigma^x[nqp, nqp] summed over k-points with compensated addition."""
    acc = _CompensatedSum((nqp, nqp))
    for z, v, wk in blocks:
        acc.add(sigx_block(z, v, wk))
    return acc.value()


def sigx_brute(blocks: Iterable[SigxBlock], nqp: int) -> np.ndarray:
    """Explicit loops over k, n', mu, n, m (tiny inputs only)."""
    out = np.zeros((nqp, nqp), np.complex128)
    for z, v, wk in blocks:
        nocc, nmu, _ = z.shape
        for a in range(nocc):
            for mu in range(nmu):
                for n in range(nqp):
                    for m in range(nqp):
                        out[n, m] -= wk * np.conj(z[a, mu, n]) * v[mu] * z[a, mu, m]
    return out


def sigx_exact(blocks, nqp: int):
    """Exact rational evaluation: Z entries as (Fraction re, Fraction im)
    pairs, v and w_k as Fractions.  Returns [nqp][nqp] of (re, im)."""
    out = [[(Fraction(0), Fraction(0)) for _ in range(nqp)] for _ in range(nqp)]
    for z, v, wk in blocks:
        nocc = len(z)
        nmu = len(z[0])
        for a in range(nocc):
            for mu in range(nmu):
                c = wk * v[mu]
                for n in range(nqp):
                    ar, ai = z[a][mu][n]
                    for m in range(nqp):
                        br, bi = z[a][mu][m]
                        # conj(a) * b = (ar br + ai bi) + i (ar bi - ai br)
                        re = ar * br + ai * bi
                        im = ar * bi - ai * br
                        r0, i0 = out[n][m]
                        out[n][m] = (r0 - c * re, i0 - c * im)
    return out


def sigx_workload_blocks(wl, q: int = 0):
    """Stream (Z, v, w_k) of a synthetic exchange workload."""
    for blk in wl.blocks(q):
        yield wl.z_block(blk), wl.coulomb(blk), blk.wk
