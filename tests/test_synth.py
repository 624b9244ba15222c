"""Seeded input generator: Philox known answers, determinism, random access,
ranges and shapes of the five workloads."""
import numpy as np
import pytest

from synth import philox4x32, workload, z_scale_table, gauss_legendre_imag_axis


def test_philox_known_answers():
    # Known-answer vectors published with Random123 for philox4x32-10.
    cases = [
        ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
        ((0xFFFFFFFF,) * 4, (0xFFFFFFFF, 0xFFFFFFFF),
         (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
        ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
         (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
    ]
    for ctr, key, want in cases:
        got = tuple(int(x) for x in philox4x32(*ctr, *key))
        assert got == want


def test_z_random_access_matches_block():
    wl = workload(0)
    blk = wl.blocks()[3]
    z = wl.z_block(blk)
    pairs = np.array([0, 5, 77, blk.npairs - 1])
    cols = np.array([0, 1, 31, 63])
    sub = wl.z_elements(blk, pairs, cols)
    flat = z.reshape(blk.npairs, wl.npb)
    assert np.array_equal(sub, flat[np.ix_(pairs, cols)])


def test_z_deterministic_and_distinct_blocks():
    wl = workload(0)
    b0, b1 = wl.blocks()[:2]
    assert np.array_equal(wl.z_block(b0), wl.z_block(b0))
    assert not np.array_equal(wl.z_block(b0), wl.z_block(b1))
    assert not np.array_equal(wl.z_block(b0), wl.replace(seed=1).z_block(b0))


def test_z_statistics_and_decay():
    wl = workload(0, npb=64, nocc=16, nunocc=64)
    z = wl.z_block(wl.blocks()[0]).reshape(-1, 64)
    f = z_scale_table(64) / z_scale_table(64)[0]
    scaled = z / f[None, :]
    assert abs(scaled.real.std() - 1) < 0.02 and abs(scaled.imag.std() - 1) < 0.02
    assert abs(scaled.real.mean()) < 0.02
    assert np.max(np.abs(scaled.real)) <= np.sqrt(3) * 2 + 1e-12


def test_c64_is_rounded_c128():
    wl64 = workload(0, ztype="c64")
    wl128 = workload(0)
    b = wl64.blocks()[0]
    z64 = wl64.z_block(b)
    assert z64.dtype == np.complex64
    assert np.array_equal(z64, wl128.z_block(b).astype(np.complex64))


def test_energy_ranges():
    for cfg in range(5):
        wl = workload(cfg)
        for blk in wl.blocks()[:4]:
            eo, eu = wl.energies(blk)
            assert eo.shape == (blk.nocc,) and eu.shape == (blk.nunocc,)
            assert np.all(np.diff(eo) >= 0) and np.all(np.diff(eu) >= 0)
            assert eo.min() >= wl.occ_range[0] and eo.max() < 0.0
            assert eu.min() >= wl.unocc_range[0] and eu.max() < wl.unocc_range[1]


def test_workload_shapes():
    assert workload(0).npairs() == 8 * 8 * 32
    assert workload(1).npairs() == 64 * 40 * 300
    assert workload(2).npairs() == 16 * 200 * 1200
    w3 = workload(3)
    sizes = [(b.nocc, b.nunocc) for q in range(w3.nq) for b in w3.blocks(q)]
    assert len(sizes) == 32 * 16
    assert min(s[0] for s in sizes) >= 16 and max(s[0] for s in sizes) <= 64
    assert min(s[1] for s in sizes) >= 100 and max(s[1] for s in sizes) <= 400
    assert len(set(sizes)) > 100
    w4 = workload(4)
    b4 = w4.blocks()
    assert len(b4) == 256 and {b.spin for b in b4} == {0, 1}
    assert all(52 <= b.nocc <= 68 and b.nunocc == 500 for b in b4)


def test_metallic_blocks_have_excluded_pairs():
    wl = workload(4)
    excl = 0
    for blk in wl.blocks()[:32]:
        eo, eu = wl.energies(blk)
        excl += int(((eu[None, :] - eo[:, None]) < wl.delta_min).sum())
    assert 16 < excl < 200   # about two per block


def test_gauss_legendre_map():
    w = gauss_legendre_imag_axis(12)
    assert np.all(np.diff(w) > 0) and w[0] > 0
    x = (w - 1) / (w + 1)
    xr, _ = np.polynomial.legendre.leggauss(12)
    assert np.allclose(np.sort(x), np.sort(xr), atol=1e-13)


def test_correlation_workload_inputs():
    """Workload 6 (imaginary-axis correlation self-energy): sizes, energies
    and the synthetic W^c (Hermitian, negative definite, decaying in w)."""
    wl = workload(6)
    assert wl.omega[0] == 0.0 and np.all(np.diff(wl.omega) > 0) and wl.nomega == 11
    blks = wl.blocks()
    assert len(blks) == 16 and all(b.nocc == 361 and b.nunocc == 1356 for b in blks)
    eq = wl.eps_qp()
    assert eq.shape == (206,) and (eq < 0).sum() == 92 and np.all(np.diff(eq) >= 0)
    em = wl.eps_mid(blks[3])
    assert em.shape == (361,) and (em < 0).sum() == 92
    small = wl.replace(npb=5, nocc=4, nunocc=24, nval=2)
    b = small.blocks()[1]
    w = small.wc_block(b)
    assert w.shape == (11, 24, 24)
    assert np.array_equal(w, np.conj(np.transpose(w, (0, 2, 1))))
    ev = np.linalg.eigvalsh(w)
    assert ev.max() < 0
    norms = np.linalg.norm(w, axis=(1, 2))
    assert np.all(np.diff(norms) < 0)
    # large-w tail ~ 1/w^2 for the first product-basis function
    assert abs(w[-1, 0, 0] / w[-2, 0, 0] - (1 + (wl.omega[-2] / 0.3) ** 2) /
               (1 + (wl.omega[-1] / 0.3) ** 2)) < 1e-12
    assert not np.array_equal(small.wc_block(small.blocks()[2]), w)
