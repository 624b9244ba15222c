"""The histogram + Hilbert oracle against its pins, and planted mistakes (on
the CPU) that the pins must catch."""
import numpy as np
import pytest

import oracle.hist_oracle as orc
import pins_hist

_bin_fractions = orc.bin_fractions
_hilbert_imag = orc.hilbert_imag
_hilbert_real = orc.hilbert_real
_hist_block = orc.hist_block


def test_hist_pins():
    res = pins_hist.run_all(orc)
    bad = {k: v for k, v in res.items() if v}
    assert not bad, bad


def _frac_left_tie(delta, edges, sigma):              # tie goes to the left bin
    if sigma == 0.0:
        e = np.asarray(edges, float)
        if delta <= e[0] or delta > e[-1]:
            return []
        return [(int(np.searchsorted(e, delta, side="left")) - 1, 1.0)]
    return _bin_fractions(delta, edges, sigma)


def _frac_one_sided(delta, edges, sigma):             # spread [D, D (1 + 2 sigma)]
    return _bin_fractions(delta * (1 + sigma), edges, sigma / (1 + sigma)) if sigma else \
        _bin_fractions(delta, edges, sigma)


def _frac_unnormalised(delta, edges, sigma):          # overlap not divided by the width
    return [(j, f * 2 * sigma * delta) if sigma else (j, f)
            for j, f in _bin_fractions(delta, edges, sigma)]


def _imag_no_width(edges, omega):
    e = np.asarray(edges, float)
    return _hilbert_imag(edges, omega) * (e[1:] - e[:-1])[None, :]


def _imag_linear(edges, omega):                       # ln(e + w) instead of ln(e^2 + w^2)
    e = np.asarray(edges, float)
    w = np.asarray(omega, float)[:, None]
    return 2 * (np.log(e[None, 1:] + w) - np.log(e[None, :-1] + w)) / (e[1:] - e[:-1])[None, :]


def _real_no_density(edges, omega):
    return np.real(_hilbert_real(edges, omega)) + 0j


def _real_density_sign(edges, omega):
    c = _hilbert_real(edges, omega)
    return np.real(c) - 1j * np.imag(c)


def _real_no_mirror(edges, omega):                    # drops the 1/(x + w) term
    e = np.asarray(edges, float)
    w = np.asarray(omega, float)[:, None]
    lo, hi = e[None, :-1], e[None, 1:]
    c = _hilbert_real(edges, omega)
    return c - (np.log(hi + w) - np.log(lo + w)) / (hi - lo)


def _block_conj_second(z, eo, eu, wk, edges, sigma, delta_min):
    return np.conj(_hist_block(z, eo, eu, wk, edges, sigma, delta_min))


def _block_positive(z, eo, eu, wk, edges, sigma, delta_min):
    return -_hist_block(z, eo, eu, wk, edges, sigma, delta_min)


@pytest.mark.parametrize("name,fn", [
    ("bin_fractions", _frac_left_tie), ("bin_fractions", _frac_one_sided),
    ("bin_fractions", _frac_unnormalised), ("hilbert_imag", _imag_no_width),
    ("hilbert_imag", _imag_linear), ("hilbert_real", _real_no_density),
    ("hilbert_real", _real_density_sign), ("hilbert_real", _real_no_mirror),
    ("hist_block", _block_conj_second), ("hist_block", _block_positive)])
def test_hist_mutation_caught(name, fn, monkeypatch):
    monkeypatch.setattr(orc, name, fn)
    res = pins_hist.run_all(orc)
    assert any(res.values()), f"{fn.__name__} not caught"
