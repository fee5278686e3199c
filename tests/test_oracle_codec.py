"""Pins of the FP16 + per-site scale emulation: the IEEE half grid and its
round-to-nearest-even rule, the error bound, and the zero site."""

import numpy as np

import synth
from oracle import codec


def test_round_trip_error_bound():
    psi = synth.gaussian_fermion((2, 2, 2, 2), 4, seed=40) * np.exp(np.random.default_rng(1).uniform(-20, 20, (4, 2, 2, 2, 2, 1, 1)))
    q, s = codec.encode(psi)
    back = codec.decode(q, s)
    err = np.abs(back - psi)
    # each real component is within half an fp16 ulp of its value relative to the site scale
    bound = (2.0**-11) * s[..., None, None] * np.sqrt(2) * (1 + 1e-6)
    assert np.all(err <= bound)
    assert np.all(np.abs(q.astype(np.float32)) <= 1.0)


def test_exact_values_and_ties():
    psi = np.zeros((1, 1, 1, 1, 1, 4, 3), dtype=np.complex128)
    # scale 2.0; in [0.5, 1) the half grid spacing is 2^-11, so 0.5 + 2^-12 and
    # 0.5 + 3 * 2^-12 are ties that round to the even neighbours 0.5 and 0.5 + 2^-10
    psi[..., 0, 0] = 2.0
    psi[..., 0, 1] = 2.0 * (0.5 + 2.0**-12)
    psi[..., 0, 2] = 2.0 * (0.5 + 3 * 2.0**-12)
    psi[..., 1, 0] = -0.5j
    q, s = codec.encode(psi)
    assert s.ravel()[0] == 2.0
    assert q[..., 0, 0, 0].ravel()[0] == np.float16(1.0)
    assert q[..., 0, 1, 0].ravel()[0] == np.float16(0.5)
    assert q[..., 0, 2, 0].ravel()[0] == np.float16(0.5 + 2.0**-10)
    assert q[..., 1, 0, 1].ravel()[0] == np.float16(-0.25)


def test_zero_site():
    psi = np.zeros((2, 1, 1, 1, 2, 4, 3), dtype=np.complex128)
    psi[1, ..., 0, :] = 1.0
    q, s = codec.encode(psi)
    assert np.all(s[0] == 0) and np.all(q[0] == 0)
    assert np.all(codec.decode(q, s)[0] == 0)
