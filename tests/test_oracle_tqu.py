"""Pins of the oracle's spin-2 harmonics and Q, U synthesis (the production
maps of Sect. 3: T, Q and U from a^T and a^E): the spin-weighted Legendre
functions against the eth operator applied to scipy's Y_lm by finite
differences, the closed form of 2Y_20, the sum rule over m, orthonormality
on the Gauss-Legendre grid, and Q - iU from the spin -2 functions."""
import math

import numpy as np
import pytest
from scipy.special import sph_harm_y

from paper_0909_0009_amd import inputs


def _lam(l, m, th):
    """lambda_lm(cos theta) with the Condon-Shortley phase, any sign of m."""
    return float(sph_harm_y(l, m, th, 0.0).real)


def _eth2(l, m, s, th, h=1e-4):
    """sY_lm / e^{i m phi} for s = +-2 by finite differences: 2Y = D^-1/2
    (d - cot - m/sin)(d - m/sin) Y and -2Y = D^-1/2 (d - cot + m/sin)(d + m/sin) Y
    (eth raising, eth-bar lowering), D = (l-1) l (l+1) (l+2)."""
    f = lambda t: _lam(l, m, t)
    d1 = (f(th + h) - f(th - h)) / (2 * h)
    d2 = (f(th + h) - 2 * f(th) + f(th - h)) / h ** 2
    sn, cs = math.sin(th), math.cos(th)
    sg = 1 if s > 0 else -1
    val = d2 - cs / sn * d1 - sg * 2 * m / sn * d1 + (sg * 2 * m * cs + m * m) / sn ** 2 * f(th)
    return val / math.sqrt((l - 1) * l * (l + 1) * (l + 2))


@pytest.mark.parametrize("s", [2, -2])
def test_spin_lambda_matches_eth_of_scipy(orc, s):
    worst = 0.0
    for x in (0.83, 0.21, -0.56):
        th = math.acos(x)
        for l in range(2, 12):
            lam = orc.spin_lambda(11, 0, s, x)  # noqa: F841 (exercise m = 0 too)
            for m in range(-l, l + 1):
                got = orc.spin_lambda(11, m, s, x)[l]
                worst = max(worst, abs(got - _eth2(l, m, s, th)))
    assert worst <= 1e-6


def test_closed_form_2Y20(orc):
    for x in (0.9, 0.1, -0.7):
        ref = 0.25 * math.sqrt(15.0 / (2.0 * math.pi)) * (1.0 - x * x)
        assert abs(orc.spin_lambda(4, 0, 2, x)[2] - ref) <= 1e-15


@pytest.mark.parametrize("s", [2, -2])
def test_sum_rule_over_m(orc, s):
    """sum_m |sY_lm|^2 = (2l+1)/(4 pi) at every point, up to l = 300."""
    L = 300
    for x in (0.999, 0.5, -0.31):
        tot = np.zeros(L + 1)
        for m in range(-L, L + 1):
            tot += orc.spin_lambda(L, m, s, x) ** 2
        ls = np.arange(2, L + 1)
        assert np.max(np.abs(tot[2:] - (2 * ls + 1) / (4 * math.pi)) / ((2 * ls + 1) / (4 * math.pi))) <= 1e-12


def test_orthonormal_on_gauss_legendre_grid(orc):
    L = 20
    x, w = orc.gl_grid(L + 1)
    for m in (-3, 0, 2, 7):
        F = np.stack([orc.spin_lambda(L, m, 2, xi) for xi in x])  # [ring][l]
        G = 2 * math.pi * (F * w[:, None]).T @ F
        l0 = max(abs(m), 2)
        ref = np.zeros_like(G)
        ref[np.arange(l0, L + 1), np.arange(l0, L + 1)] = 1.0
        assert np.max(np.abs(G - ref)) <= 1e-13


def test_qu_maps_single_modes_and_conjugate_spin(orc):
    """aE = c at (2, 0): Q = -c 2Y_20, U = 0.  For a random field, Q - iU
    from the spin -2 functions (-sum aE -2Y) equals conj(Q + iU)."""
    L, nphi = 6, 19
    x = np.array([0.93, 0.4, -0.2, -0.88])
    a = np.zeros(inputs.nlm(L), dtype=complex)
    a[inputs.lm_arrays(L)[0].tolist().index(2)] = 1.5
    Q, U = orc.synth_qu(L, x, nphi, a)
    ref = -1.5 * 0.25 * math.sqrt(15 / (2 * math.pi)) * (1 - x * x)
    assert np.max(np.abs(Q - ref[:, None])) <= 1e-14 and np.max(np.abs(U)) <= 1e-14
    rng = np.random.default_rng(4)
    a = rng.standard_normal(inputs.nlm(L)) + 1j * rng.standard_normal(inputs.nlm(L))
    ls, ms = inputs.lm_arrays(L)
    a[ms == 0] = a[ms == 0].real
    a[ls < 2] = 0
    Q, U = orc.synth_qu(L, x, nphi, a)
    phi = 2 * math.pi * np.arange(nphi) / nphi
    qmu = np.zeros((x.size, nphi), dtype=complex)
    for k, xi in enumerate(x):
        for m in range(-L, L + 1):
            lam = orc.spin_lambda(L, m, -2, xi)
            for l in range(max(2, abs(m)), L + 1):
                v = a[l * (l + 1) // 2 + abs(m)]
                if m < 0:
                    v = (-1) ** m * np.conj(v)
                qmu[k] -= v * lam[l] * np.exp(1j * m * phi)
    assert np.max(np.abs(qmu - (Q - 1j * U))) <= 1e-13 * np.max(np.abs(Q))
