"""The oracle on hypothesis-drawn small inputs (CPU): the loop tier equals the
reference tier, and the structural facts of the polarization hold for any
shape -- Hermitian, negative semidefinite, Loewner-monotone in the imaginary
frequency (|f| = 2D / (D^2 + w^2) decreases in w), additive over blocks and
unchanged by a phase on each pair's row.  Inputs with D <= 0 pairs are
rejected unless skipping them is asked for."""
import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle

U = np.finfo(float).eps


@st.composite
def small(draw):
    npb = draw(st.integers(1, 12))
    blocks = draw(st.lists(st.tuples(st.integers(0, 3), st.integers(0, 5)), min_size=1, max_size=3))
    seed = draw(st.integers(0, 2 ** 31 - 1))
    rng = np.random.default_rng(seed)
    out = []
    for nocc, nunocc in blocks:
        z = rng.standard_normal((nocc, nunocc, npb)) + 1j * rng.standard_normal((nocc, nunocc, npb))
        eo = -rng.uniform(0.05, 1.0, nocc)
        eu = rng.uniform(-0.1, 1.5, nunocc)            # some D <= 0: skipped
        out.append((z, eo, eu, float(rng.uniform(0.1, 1.0))))
    omega = np.sort(rng.uniform(0.0, 3.0, 3))
    dmin = float(draw(st.sampled_from([0.0, 0.05, 0.3])))
    return out, npb, omega, dmin, rng


@settings(max_examples=40, deadline=None, derandomize=True, database=None)
@given(small())
def test_oracle_structure(case):
    blocks, npb, omega, dmin, rng = case
    # D <= 0 pairs, counted by hand: rejected in strict mode, skipped otherwise
    bad = sum(1 for _, eo, eu, _ in blocks for o in eo for u in eu if not u - o > 0)
    assert sum(oracle.nonpositive_pairs(eo, eu) for _, eo, eu, _ in blocks) == bad
    if bad:
        with pytest.raises(oracle.InvalidPairs):
            oracle.chi0_ref(blocks, npb, omega, dmin)
        with pytest.raises(oracle.InvalidPairs):
            oracle.chi0_brute(blocks, npb, omega, dmin)
    ref = oracle.chi0_ref(blocks, npb, omega, dmin, strict=False)
    scale = max(1.0, float(np.abs(ref).max()))
    # loop tier == reference tier
    assert np.abs(oracle.chi0_brute(blocks, npb, omega, dmin, strict=False) - ref).max() <= 1e-13 * scale
    for iw in range(len(omega)):
        c = ref[iw]
        assert np.abs(c - c.conj().T).max() <= 1e-14 * scale           # Hermitian
        assert np.linalg.eigvalsh(c).max() <= 64 * U * scale * npb     # negative semidefinite
    for a, b in zip(ref[:-1], ref[1:]):                                # omega ascending
        assert np.linalg.eigvalsh(b - a).min() >= -64 * U * scale * npb  # chi0(w1) <= chi0(w2)
    # additive over blocks
    parts = sum(oracle.chi0_ref([blk], npb, omega, dmin, strict=False) for blk in blocks)
    assert np.abs(parts - ref).max() <= 1e-13 * scale
    # a phase on each pair's row changes nothing
    rot = [(z * np.exp(1j * rng.uniform(0, 2 * np.pi, z.shape[:2]))[..., None], eo, eu, wk)
           for z, eo, eu, wk in blocks]
    assert np.abs(oracle.chi0_ref(rot, npb, omega, dmin, strict=False) - ref).max() <= 1e-13 * scale
