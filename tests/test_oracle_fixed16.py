"""Pins of the oracle's 16-bit fixed-point storage format (the "half" format
of Section V): the round-trip error bound that follows from rounding to
codes of step m / 32767, the extreme codes, zero sites, and the
per-site independence of the norm (CPU only)."""
import numpy as np

import oracle
import synth


def test_round_trip_within_half_a_code_step():
    """|v - read(store(v))| <= (1/2 + 2^-6) m / 32767 for every real of a
    site with norm m: half a code step from the rounding to a code, plus the
    FP32 roundings of the scaled value and of the read-back (four roundings
    of relative size 2^-24 on values of up to 32767 steps: below 2^-7 of a
    step)."""
    psi = synth.gaussian_spinor((4, 4, 4, 4), 31) * np.exp(np.random.default_rng(32).normal(size=(4, 4, 4, 4, 1, 1)))
    back = oracle.fixed16_site_round(psi)
    r = np.stack([psi.real, psi.imag], -1).reshape(-1, 24)
    b = np.stack([back.real, back.imag], -1).reshape(-1, 24)
    m = np.abs(r).max(axis=1, keepdims=True)
    assert np.all(np.abs(r - b) <= (0.5 + 2.0 ** -6) * m / 32767.0)
    # and not trivially: the error reaches a good part of the bound somewhere
    assert np.max(np.abs(r - b) / (m / 32767.0)) > 0.4


def test_largest_element_and_codes():
    """The largest magnitude of a site takes code +-32767 and reads back as
    +-m to FP32 accuracy; codes never leave [-32767, 32767]."""
    v = np.random.default_rng(5).normal(size=(1000, 24)) * 10.0 ** np.random.default_rng(6).uniform(-3, 3, (1000, 1))
    q, m = oracle.fixed16_codes(v, 1)
    assert q.min() >= -32767 and q.max() <= 32767
    k = np.argmax(np.abs(v), axis=1)
    assert np.all(np.abs(q[np.arange(1000), k]) == 32767)
    back = oracle.fixed16_decode(q, m)
    assert np.allclose(np.abs(back[np.arange(1000), k]), np.abs(v[np.arange(1000), k]), rtol=2e-7, atol=0)


def test_zero_site_and_scale_invariance():
    """A zero site stays exactly zero, and scaling one site by a power of two
    scales its read-back values exactly without touching other sites."""
    v = np.random.default_rng(7).normal(size=(3, 24))
    v[1] = 0.0
    q, m = oracle.fixed16_codes(v, 1)
    back = oracle.fixed16_decode(q, m)
    assert np.all(back[1] == 0.0) and m[1, 0] == 0.0
    v2 = v.copy()
    v2[2] *= 8.0
    q2, m2 = oracle.fixed16_codes(v2, 1)
    b2 = oracle.fixed16_decode(q2, m2)
    assert np.array_equal(q2, q) and np.array_equal(b2[2], 8.0 * back[2]) and np.array_equal(b2[0], back[0])
