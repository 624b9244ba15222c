"""The exchange self-energy oracle against its pins, and planted mistakes
(on the CPU) that the pins must catch."""
import numpy as np
import pytest

import oracle.sigx_oracle as orc
import pins_sigx


def test_sigx_pins():
    res = pins_sigx.run_all(orc)
    bad = {k: v for k, v in res.items() if v}
    assert not bad, bad


def _block_repeat(z, v, wk):          # v indexed by n' instead of mu
    z = np.asarray(z)
    nocc, nmu, nqp = z.shape
    a = z.reshape(nocc * nmu, nqp).astype(np.complex128)
    c = np.repeat(np.asarray(v, np.float64), nocc)[: nocc * nmu] * wk
    return -(a.conj().T @ (c[:, None] * a))


def _block_conj_second(z, v, wk):     # conjugation on the second state
    z = np.asarray(z)
    nocc, nmu, nqp = z.shape
    a = z.reshape(nocc * nmu, nqp).astype(np.complex128)
    c = np.tile(np.asarray(v, np.float64), nocc) * wk
    return -(a.T @ (c[:, None] * a.conj()))


def _block_no_minus(z, v, wk):
    z = np.asarray(z)
    nocc, nmu, nqp = z.shape
    a = z.reshape(nocc * nmu, nqp).astype(np.complex128)
    return a.conj().T @ ((np.tile(v, nocc) * wk)[:, None] * a)


def _block_sqrt_v(z, v, wk):
    z = np.asarray(z)
    nocc, nmu, nqp = z.shape
    a = z.reshape(nocc * nmu, nqp).astype(np.complex128)
    return -(a.conj().T @ ((np.tile(np.sqrt(v), nocc) * wk)[:, None] * a))


def _block_no_wk(z, v, wk):
    z = np.asarray(z)
    nocc, nmu, nqp = z.shape
    a = z.reshape(nocc * nmu, nqp).astype(np.complex128)
    return -(a.conj().T @ (np.tile(v, nocc)[:, None] * a))


@pytest.mark.parametrize("fn", [_block_repeat, _block_conj_second, _block_no_minus,
                                _block_sqrt_v, _block_no_wk])
def test_sigx_mutation_caught(fn, monkeypatch):
    monkeypatch.setattr(orc, "sigx_block", fn)
    res = pins_sigx.run_all(orc)
    assert any(res.values()), f"{fn.__name__} not caught"
