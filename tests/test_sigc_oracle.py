"""The imaginary-axis correlation self-energy oracle against its pins, and
planted mistakes (on the CPU) that the pins must catch."""
import mpmath
import numpy as np
import pytest

import oracle.sigc_oracle as orc
import pins_sigc

_ag_weights = orc.ag_weights


def test_sigc_pins():
    res = pins_sigc.run_all(orc)
    bad = {k: v for k, v in res.items() if v}
    assert not bad, bad


# ---------------------------------------------------------- planted mistakes
def _block_weight_on_m(z, wc, weights, wk):        # weight follows column m
    z = np.asarray(z, np.complex128)
    out = np.zeros((z.shape[2], z.shape[2]), np.complex128)
    for a in range(z.shape[0]):
        for i in range(wc.shape[0]):
            out += z[a].conj().T @ wc[i] @ (z[a] * weights[a, :, i][None, :])
    return -wk * out


def _block_conj_second(z, wc, weights, wk):
    z = np.asarray(z, np.complex128)
    out = np.zeros((z.shape[2], z.shape[2]), np.complex128)
    for a in range(z.shape[0]):
        for i in range(wc.shape[0]):
            out += (z[a] * weights[a, :, i][None, :]).T @ wc[i] @ z[a].conj()
    return -wk * out


def _block_no_minus(z, wc, weights, wk):
    return -orc_block(z, wc, weights, wk)


def _block_w_transposed(z, wc, weights, wk):
    return orc_block(z, np.transpose(wc, (0, 2, 1)), weights, wk)


def _block_no_wk(z, wc, weights, wk):
    return orc_block(z, wc, weights, 1.0)


orc_block = orc.sigc_block


def _weights_no_tail(delta, mesh):
    w = _ag_weights(delta, mesh)
    if delta == 0:
        return w
    c = mesh[-1]
    t = abs(delta) / c
    w[-1] -= np.sign(delta) * (t - np.arctan(t)) / t ** 2 / np.pi
    return w


def _weights_no_flat(delta, mesh):
    w = _ag_weights(delta, mesh)
    if delta != 0:
        w[0] -= np.arctan(mesh[0] / delta) / np.pi
    return w


def _weights_swapped_hats(delta, mesh):
    """Each interval's two hat-function halves given to the wrong node."""
    mesh = [float(x) for x in mesh]
    n = len(mesh)
    if delta == 0 or n < 2:
        return _ag_weights(delta, mesh)
    w = _ag_weights(delta, mesh)
    with mpmath.workdps(40):
        d = mpmath.mpf(delta)
        for j in range(n - 1):
            a, b = mpmath.mpf(mesh[j]), mpmath.mpf(mesh[j + 1])
            i0 = mpmath.atan(b / d) - mpmath.atan(a / d)
            i1 = d / 2 * (mpmath.log(d * d + b * b) - mpmath.log(d * d + a * a))
            left = float((b * i0 - i1) / (b - a) / mpmath.pi)
            right = float((i1 - a * i0) / (b - a) / mpmath.pi)
            w[j] += right - left
            w[j + 1] += left - right
    return w


def _weights_no_pi(delta, mesh):
    return _ag_weights(delta, mesh) * np.pi


def _table_sign_flipped(eps_qp, eps_mid, mesh):     # dE = eps_mid - eps_qp
    out = np.empty((len(eps_mid), len(eps_qp), len(mesh)))
    for a, e1 in enumerate(eps_mid):
        for n, e0 in enumerate(eps_qp):
            out[a, n] = _ag_weights(float(e1 - e0), mesh)
    return out


@pytest.mark.parametrize("fn", [_block_weight_on_m, _block_conj_second, _block_no_minus,
                                _block_w_transposed, _block_no_wk])
def test_sigc_block_mutation_caught(fn, monkeypatch):
    monkeypatch.setattr(orc, "sigc_block", fn)
    res = pins_sigc.run_all(orc)
    assert any(res.values()), f"{fn.__name__} not caught"


@pytest.mark.parametrize("fn", [_weights_no_tail, _weights_no_flat, _weights_swapped_hats,
                                _weights_no_pi])
def test_sigc_weight_mutation_caught(fn, monkeypatch):
    monkeypatch.setattr(orc, "ag_weights", fn)
    res = pins_sigc.run_all(orc)
    assert any(res.values()), f"{fn.__name__} not caught"


def test_sigc_sign_mutation_caught(monkeypatch):
    monkeypatch.setattr(orc, "ag_weight_table", _table_sign_flipped)
    res = pins_sigc.run_all(orc)
    assert any(res.values()), "energy-difference sign not caught"
