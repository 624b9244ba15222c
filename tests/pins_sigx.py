"""Pins of the exchange self-energy oracle (oracle/sigx_oracle.py) against
what Eq.(sigx) and linear algebra fix: a hand-derived example, exact rational
arithmetic, explicit loops, the rank-one closed form, Hermiticity and
negative semidefiniteness, and structural identities."""
import json
import os
from fractions import Fraction

import numpy as np

U = np.finfo(np.float64).eps / 2
HERE = os.path.dirname(os.path.abspath(__file__))


def _close(a, b, tol):
    a = np.asarray(a)
    b = np.asarray(b)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


def _golden():
    with open(os.path.join(HERE, "golden", "sigx_two_state_example.json")) as f:
        g = json.load(f)
    z = np.array([[[complex(r, i) for r, i in row] for row in blk] for blk in g["z"]])
    v = np.array([float(Fraction(x)) for x in g["v"]])
    ref = np.array([[complex(float(Fraction(r)), float(Fraction(i))) for r, i in row]
                    for row in g["sigx"]])
    return g, z, v, float(Fraction(g["wk"])), ref


def pin_golden(orc):
    fails = []
    g, z, v, wk, ref = _golden()
    got = orc.sigx_ref([(z, v, wk)], 2)
    if not _close(got, ref, 1e-15):
        fails.append(f"golden sigx: {got}")
    ev = np.linalg.eigvalsh(got)
    if not _close(ev, [float(Fraction(x)) for x in g["eigenvalues"]], 1e-14):
        fails.append(f"golden eigenvalues: {ev}")
    return fails


def pin_exact_and_brute(orc):
    """Small-integer Z, dyadic v and w_k: exact rational result = explicit
    loops = reference (two blocks, nocc and nmu both > 1)."""
    fails = []
    rng = np.random.default_rng(11)
    nqp = 3
    blocks, exact_in = [], []
    for nocc, nmu, wk in ((2, 3, Fraction(1, 2)), (3, 2, Fraction(1, 4))):
        zr = rng.integers(-3, 4, (nocc, nmu, nqp))
        zi = rng.integers(-3, 4, (nocc, nmu, nqp))
        v = [Fraction(int(x), 8) for x in rng.integers(1, 9, nmu)]
        blocks.append((zr + 1j * zi, np.array([float(x) for x in v]), float(wk)))
        exact_in.append(([[[(Fraction(int(zr[a, m, n])), Fraction(int(zi[a, m, n])))
                            for n in range(nqp)] for m in range(nmu)] for a in range(nocc)],
                         v, wk))
    ex = orc.sigx_exact(exact_in, nqp)
    ex = np.array([[float(r) + 1j * float(i) for r, i in row] for row in ex])
    if not _close(orc.sigx_brute(blocks, nqp), ex, 1e-15):
        fails.append("brute vs exact")
    if not _close(orc.sigx_ref(blocks, nqp), ex, 1e-15):
        fails.append("ref vs exact")
    return fails


def pin_rank_one(orc):
    """One k-point, one occupied state, one product-basis function:
    Sigma^x = -w_k v conj(z) z^T."""
    fails = []
    rng = np.random.default_rng(3)
    z = rng.standard_normal(5) + 1j * rng.standard_normal(5)
    got = orc.sigx_ref([(z.reshape(1, 1, 5), np.array([0.7]), 0.25)], 5)
    if not _close(got, -0.25 * 0.7 * np.outer(z.conj(), z), 4e-16):
        fails.append("rank one")
    return fails


def pin_invariants(orc):
    """Hermitian, negative semidefinite, rank <= rows; additivity over
    k-points; permutations of n' and of mu (with v); per-row phases; v -> a v
    and w_k -> b w_k scale the result."""
    fails = []
    rng = np.random.default_rng(5)
    nqp = 7
    blocks = []
    for nocc, nmu in ((2, 2), (1, 3)):
        z = rng.standard_normal((nocc, nmu, nqp)) + 1j * rng.standard_normal((nocc, nmu, nqp))
        blocks.append((z, rng.uniform(0.1, 2.0, nmu), rng.uniform(0.2, 1.0)))
    s = orc.sigx_ref(blocks, nqp)
    if not _close(s, s.conj().T, 1e-15):
        fails.append("not Hermitian")
    ev = np.linalg.eigvalsh(s)
    scale = np.max(np.abs(ev))
    if ev.max() > 64 * U * scale:
        fails.append(f"not NSD: {ev.max()}")
    if np.sum(np.abs(ev) > 1e-10 * scale) > 4 + 3:
        fails.append("rank above the number of rows")
    parts = sum(orc.sigx_ref([b], nqp) for b in blocks)
    if not _close(parts, s, 1e-14):
        fails.append("additivity")
    z, v, wk = blocks[0]
    po, pm = np.array([1, 0]), np.array([1, 0])
    perm = orc.sigx_ref([(z[po][:, pm], v[pm], wk), blocks[1]], nqp)
    if not _close(perm, s, 1e-14):
        fails.append("permutation of n' / mu")
    ph = np.exp(1j * rng.uniform(0, 2 * np.pi, (2, 2, 1)))
    if not _close(orc.sigx_ref([(z * ph, v, wk), blocks[1]], nqp), s, 1e-14):
        fails.append("per-row phase")
    if not _close(orc.sigx_ref([(z, 3 * v, 2 * wk)], nqp), 6 * orc.sigx_ref([blocks[0]], nqp),
                  1e-14):
        fails.append("scaling of v and w_k")
    return fails


ALL_PINS = [pin_golden, pin_exact_and_brute, pin_rank_one, pin_invariants]


def run_all(orc):
    out = {}
    for p in ALL_PINS:
        try:
            out[p.__name__] = p(orc)
        except Exception as exc:  # a planted mistake may also raise
            out[p.__name__] = [f"raised {type(exc).__name__}: {exc}"]
    return out
