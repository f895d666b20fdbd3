"""Counter-based noise of the oracle (regenerated from a seed, the paper's
memory remark in Sect. 3): the Philox4x32-10 generator against its published
known-answer vectors, and the Gaussian noise against the statistics the
method assumes (Sect. 2: complex unit Gaussian, real for m = 0)."""
import os

import numpy as np

from oracle import fnl_oracle as orc

HERE = os.path.dirname(os.path.abspath(__file__))


def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        v = [int(x, 16) for x in r]
        got = orc.philox4x32_10(v[0:4], v[4:6])
        assert [int(x) for x in got] == v[6:10], r


def test_noise_is_a_function_of_the_seed():
    a = orc.seeded_noise(24, 7, 99)
    b = orc.seeded_noise(24, 7, 99)
    c = orc.seeded_noise(24, 7, 100)
    assert np.array_equal(a, b)
    assert not np.any(a == c)
    # one shell's values do not depend on how many shells are drawn
    assert np.array_equal(orc.seeded_noise(24, 3, 99), a[:3])


def test_noise_statistics():
    L, N = 96, 64
    n = orc.seeded_noise(L, N, 2024)
    l = np.repeat(np.arange(L + 1), np.arange(1, L + 2))
    m = np.arange(l.size) - l * (l + 1) // 2
    m0 = m == 0
    assert np.all(n[:, m0].imag == 0.0)
    k = n.size                                  # ~3e5 samples
    tol = 6.0 / np.sqrt(k)                      # 6 sigma of a unit-variance mean
    e2 = np.mean(np.abs(n) ** 2)
    assert abs(e2 - 1.0) < 6.0 * np.sqrt(2.0 / k), e2
    assert abs(np.mean(n.real)) < tol and abs(np.mean(n.imag)) < tol
    re, im = n[:, ~m0].real.ravel(), n[:, ~m0].imag.ravel()
    assert abs(np.var(re) - 0.5) < 0.01 and abs(np.var(im) - 0.5) < 0.01
    assert abs(np.mean(re * im)) < tol
    # Gaussian shape: P(|x| < sigma) = 0.6827, P(|x| < 2 sigma) = 0.9545
    z = np.concatenate([re, im]) / np.sqrt(0.5)
    assert abs(np.mean(np.abs(z) < 1.0) - 0.6827) < 0.005
    assert abs(np.mean(np.abs(z) < 2.0) - 0.9545) < 0.003
    # neighbouring shells and coefficients are uncorrelated
    assert abs(np.mean(n[0].real * n[1].real)) < 0.02
    assert abs(np.mean(n[:, 5:-1].real * n[:, 6:].real)) < 0.01
