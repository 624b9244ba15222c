"""Plant plausible mistakes in the oracle (on the CPU) and check that at
least one pin catches each of them."""
import numpy as np
import pytest

import oracle.chi0_oracle as orc
import pins


def _weight_sign(delta, omega, wk):
    d = np.asarray(delta, np.float64)
    return 2.0 * wk * d / (d * d + omega * omega)


def _weight_no_two(delta, omega, wk):
    d = np.asarray(delta, np.float64)
    return -wk * d / (d * d + omega * omega)


def _weight_minus_omega2(delta, omega, wk):
    d = np.asarray(delta, np.float64)
    return -2.0 * wk * d / (d * d - omega * omega + 1e-300)


def _weight_wk_twice(delta, omega, wk):
    d = np.asarray(delta, np.float64)
    return -2.0 * wk * wk * d / (d * d + omega * omega)


def _delta_transposed(eps_occ, eps_unocc):
    return np.asarray(eps_occ)[:, None] - np.asarray(eps_unocc)[None, :]


def _included_strict(delta, delta_min):
    return (delta > 0.0) & (delta > delta_min)


def _block_conj_second(z, eps_occ, eps_unocc, wk, omega, delta_min, strict=True):
    z = np.asarray(z)
    nocc, nunocc, npb = z.shape
    a = z.reshape(nocc * nunocc, npb).astype(np.complex128)
    delta = orc.pair_delta(eps_occ, eps_unocc).reshape(-1)
    keep = orc.pair_included(delta, delta_min)
    a, delta = a[keep], delta[keep]
    out = np.empty((len(omega), npb, npb), np.complex128)
    for iw, w in enumerate(omega):
        c = orc.transition_weight(delta, float(w), wk)
        out[iw] = a.T @ (c[:, None] * a.conj())
    return out



def _entries_variant(conj_second=False, no_mask=False, no_wk=False, ignore_map=False):
    """chi0_entries with one planted mistake."""
    def fn(block_columns, entries, col_index, omega, delta_min=0.0, strict=True):
        acc = orc._CompensatedSum((len(omega), len(entries)))
        cmap = (lambda i: i) if ignore_map else (lambda i: col_index[i])
        ii = np.array([cmap(i) for i, _ in entries])
        jj = np.array([cmap(j) for _, j in entries])
        for zc, eo, eu, wk in block_columns:
            orc._check_pairs(eo, eu, strict)
            delta = orc.pair_delta(eo, eu).reshape(-1)
            keep = np.ones_like(delta, bool) if no_mask else orc.pair_included(delta, delta_min)
            zc = np.asarray(zc, np.complex128)[keep]
            delta = delta[keep]
            part = np.empty((len(omega), len(entries)), np.complex128)
            for iw, w in enumerate(omega):
                c = orc.transition_weight(delta, float(w), 1.0 if no_wk else wk)
                a, b = zc[:, ii], zc[:, jj]
                part[iw] = np.sum(c[:, None] * (a * b.conj() if conj_second else a.conj() * b), axis=0)
            acc.add(part)
        return acc.value()
    return fn


def _rows_variant(conj_cols=False, rows_as_cols=False, no_wk=False):
    """chi0_rows with one planted mistake."""
    def fn(blocks, rows, npb, omega, delta_min=0.0, strict=True):
        rows = np.asarray(rows)
        acc = orc._CompensatedSum((len(omega), len(rows), npb))
        for z, eo, eu, wk in blocks:
            orc._check_pairs(eo, eu, strict)
            z = np.asarray(z)
            a = z.reshape(-1, npb).astype(np.complex128)
            delta = orc.pair_delta(eo, eu).reshape(-1)
            keep = orc.pair_included(delta, delta_min)
            a, delta = a[keep], delta[keep]
            part = np.empty((len(omega), len(rows), npb), np.complex128)
            for iw, w in enumerate(omega):
                c = orc.transition_weight(delta, float(w), 1.0 if no_wk else wk)
                if conj_cols:
                    part[iw] = a[:, rows].T @ (c[:, None] * a.conj())
                elif rows_as_cols:
                    part[iw] = (a.conj().T @ (c[:, None] * a[:, rows])).T
                else:
                    part[iw] = a[:, rows].conj().T @ (c[:, None] * a)
            acc.add(part)
        return acc.value()
    return fn


def _dielectric_plus(chi0, vsqrt):
    s = np.asarray(vsqrt)
    return np.eye(s.shape[0])[None] + s[None, :, None] * chi0 * s[None, None, :]


def _dielectric_one_side(chi0, vsqrt):
    s = np.asarray(vsqrt)
    return np.eye(s.shape[0])[None] - (s * s)[None, :, None] * chi0


def _gj_no_pivot(a):
    a = np.array(a, dtype=np.complex128)
    n = a.shape[0]
    aug = np.concatenate([a, np.eye(n, dtype=np.complex128)], axis=1)
    for k in range(n):
        aug[k] = aug[k] / aug[k, k]
        col = aug[:, k].copy()
        col[k] = 0.0
        aug -= col[:, None] * aug[k][None, :]
    return aug[:, n:]


def _chol_no_conj(a):
    """Cholesky factor with the conjugation of the row dropped."""
    a = np.array(a, dtype=np.complex128)
    n = a.shape[0]
    low = np.zeros_like(a)
    for j in range(n):
        d = a[j, j].real - np.sum(np.abs(low[j, :j]) ** 2)
        if not d > 0.0:
            raise orc.NotHPD(f"pivot {j}")
        low[j, j] = np.sqrt(d)
        low[j + 1:, j] = (a[j + 1:, j] - low[j + 1:, :j] @ low[j, :j]) / low[j, j]
    return low


def _chol_upper_read(a):
    """Cholesky factor reading the upper triangle as if it were the lower."""
    return orc.__dict__["_orig_cholesky_lower"](np.array(a).T)


def _wc_no_minus_one(eps_inv, vsqrt):
    s = np.asarray(vsqrt)
    d = np.asarray(eps_inv)
    return s[..., :, None] * d * s[..., None, :]


def _ref_drop_last_block(blocks, npb, omega, delta_min=0.0, strict=True):
    blocks = list(blocks)
    acc = orc._CompensatedSum((len(omega), npb, npb))
    for z, eo, eu, wk in blocks[:-1] if len(blocks) > 1 else blocks:
        acc.add(orc.chi0_block(z, eo, eu, wk, omega, delta_min, strict))
    return acc.value()


MUTATIONS = {
    "weight_sign": ("transition_weight", _weight_sign),
    "weight_no_two": ("transition_weight", _weight_no_two),
    "weight_minus_omega2": ("transition_weight", _weight_minus_omega2),
    "weight_wk_twice": ("transition_weight", _weight_wk_twice),
    "delta_transposed": ("pair_delta", _delta_transposed),
    "tie_excluded": ("pair_included", _included_strict),
    "conj_second_index": ("chi0_block", _block_conj_second),
    "dielectric_plus": ("dielectric", _dielectric_plus),
    "dielectric_one_side": ("dielectric", _dielectric_one_side),
    "gj_no_pivot": ("inverse_gauss_jordan", _gj_no_pivot),
    "chol_no_conj": ("cholesky_lower", _chol_no_conj),
    "chol_upper_read": ("cholesky_lower", _chol_upper_read),
    "wc_no_minus_one": ("screened_wc", _wc_no_minus_one),
    "drop_last_block": ("chi0_ref", _ref_drop_last_block),
    "entries_conj_second": ("chi0_entries", _entries_variant(conj_second=True)),
    "entries_no_mask": ("chi0_entries", _entries_variant(no_mask=True)),
    "entries_no_wk": ("chi0_entries", _entries_variant(no_wk=True)),
    "entries_ignore_col_map": ("chi0_entries", _entries_variant(ignore_map=True)),
    "rows_conj_columns": ("chi0_rows", _rows_variant(conj_cols=True)),
    "rows_are_columns": ("chi0_rows", _rows_variant(rows_as_cols=True)),
    "rows_no_wk": ("chi0_rows", _rows_variant(no_wk=True)),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, monkeypatch):
    attr, fn = MUTATIONS[name]
    monkeypatch.setattr(orc, "_orig_cholesky_lower", orc.cholesky_lower, raising=False)
    monkeypatch.setattr(orc, attr, fn)
    res = pins.run_all(orc)
    caught = [k for k, v in res.items() if v]
    assert caught, f"mutation {name} not caught by any pin"
